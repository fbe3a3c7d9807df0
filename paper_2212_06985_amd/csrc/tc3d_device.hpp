// Device-side helpers: lattice index arithmetic and the Philox4x32-10 block
// function. Conventions are those documented in include/tc3d.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc3d {

// Coordinates of a site index v = x + L*(y + L*z).
struct Coord {
    int x, y, z;
};

__device__ __forceinline__ Coord coord_of(int v, int L) {
    Coord c;
    c.x = v % L;
    int r = v / L;
    c.y = r % L;
    c.z = r / L;
    return c;
}

__device__ __forceinline__ int site_of(int x, int y, int z, int L) { return x + L * (y + L * z); }
__device__ __forceinline__ int inc(int c, int L) { return c + 1 == L ? 0 : c + 1; }
__device__ __forceinline__ int dec(int c, int L) { return c == 0 ? L - 1 : c - 1; }

// Site v shifted by +1 (dir=+1) or -1 (dir=-1) along axis a.
__device__ __forceinline__ int shift(Coord c, int a, int dir, int L) {
    if (a == 0) c.x = dir > 0 ? inc(c.x, L) : dec(c.x, L);
    else if (a == 1) c.y = dir > 0 ? inc(c.y, L) : dec(c.y, L);
    else c.z = dir > 0 ? inc(c.z, L) : dec(c.z, L);
    return site_of(c.x, c.y, c.z, L);
}

// The two axes spanning a face with normal n, in increasing order.
__device__ __forceinline__ int span_a(int n) { return n == 0 ? 1 : 0; }
__device__ __forceinline__ int span_b(int n) { return n == 2 ? 1 : 2; }

// Member edges of face f(v,n), in the documented order k = 0..3.
__device__ __forceinline__ void face_members(int n, Coord c, int L, int N, int m[4]) {
    const int a = span_a(n), b = span_b(n);
    const int v = site_of(c.x, c.y, c.z, L);
    m[0] = a * N + v;
    m[1] = a * N + shift(c, b, +1, L);
    m[2] = b * N + v;
    m[3] = b * N + shift(c, a, +1, L);
}

// The four faces containing edge e(v,a): for each other axis d, with n the
// third axis, faces f(v,n) and f(v - unit(d), n).
__device__ __forceinline__ void edge_faces(int a, Coord c, int L, int N, int f[4]) {
    const int v = site_of(c.x, c.y, c.z, L);
    int j = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == a) continue;
        const int n = 3 - a - d;
        f[j++] = n * N + v;
        f[j++] = n * N + shift(c, d, -1, L);
    }
}

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; a round
// multiplies words 0 and 2 by the round multipliers, crosses the high halves
// with words 1 and 3 and the key, and the key advances by the Weyl constants.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        U4 o;
        o.x = hi1 ^ c.y ^ k0;
        o.y = lo1;
        o.z = hi0 ^ c.w ^ k1;
        o.w = lo0;
        c = o;
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// 64 Bernoulli bits, one per shot of global word gw: shot s = 64 gw + i uses
// word (s mod 4) of the block at counter (row, cycle, s div 4, tag).
__device__ __forceinline__ uint64_t bernoulli_word(uint32_t row, uint32_t cycle, uint64_t gw,
                                                   uint32_t tag, uint32_t th, uint32_t k0,
                                                   uint32_t k1) {
    uint64_t bits = 0;
    const uint32_t base = (uint32_t)(gw * 16u);
#pragma unroll 4
    for (uint32_t j = 0; j < 16; ++j) {
        const U4 r = philox4x32_10(U4{row, cycle, base + j, tag}, k0, k1);
        const uint64_t nib = (uint64_t)(r.x < th) | ((uint64_t)(r.y < th) << 1) |
                             ((uint64_t)(r.z < th) << 2) | ((uint64_t)(r.w < th) << 3);
        bits |= nib << (4 * j);
    }
    return bits;
}

// The 64 p-flip coins of global word gw: r0 | r1 << 32 of the block at counter
// (edge, cycle, gw, 2 + sweep).
__device__ __forceinline__ uint64_t coin_word(uint32_t edge, uint32_t cycle, uint64_t gw,
                                              uint32_t sweep, uint32_t k0, uint32_t k1) {
    const U4 r = philox4x32_10(U4{edge, cycle, (uint32_t)gw, 2u + sweep}, k0, k1);
    return (uint64_t)r.x | ((uint64_t)r.y << 32);
}

}  // namespace tc3d
