// Exact uint64 arithmetic of the DP with the overflow rule: every result is
// the residue mod 2^64, and a flag records whether the exact value reached
// 2^64; and the arithmetic modulo p = 2^w - c of the residue passes.  Written
// for the device; plain C++ otherwise, so a host compiler can check it against
// 128-bit arithmetic (include it after the HIP runtime header on the device
// side).
#pragma once

#include <cstdint>

namespace sc {
namespace kern {

// acc + a*b mod 2^64; sets `ovf` when a*b >= 2^64 (the high half of the
// 128-bit product is non-zero) or the sum carries.
__host__ __device__ __forceinline__ uint64_t mad_ovf(uint64_t acc, uint64_t a, uint64_t b,
                                                     uint32_t &ovf) {
    const unsigned __int128 p = (unsigned __int128)a * b;
    const uint64_t lo = (uint64_t)p;
    const uint64_t s = acc + lo;
    ovf |= (uint32_t)((uint64_t)(p >> 64) != 0) | (uint32_t)(s < lo);
    return s;
}

// The same result with three 32-bit multiplies instead of the full 128-bit
// product; fewer vector-ALU cycles, more registers and selects.
//
// With a = ah*2^32 + al and b = bh*2^32 + bl:
//   a*b = ah*bh*2^64 + (ah*bl + al*bh)*2^32 + al*bl.
// If ah and bh are both non-zero the product is at least 2^64.  Otherwise at
// most one cross term c is non-zero and a*b = c*2^32 + al*bl, which reaches
// 2^64 exactly when c >= 2^32 or lo32(c) + hi32(al*bl) >= 2^32.  The residue
// needs only the low 32 bits of the two cross terms.
__host__ __device__ __forceinline__ uint64_t mad_ovf3(uint64_t acc, uint64_t a, uint64_t b,
                                                      uint32_t &ovf) {
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
    const uint32_t bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    const uint64_t ll = (uint64_t)al * bl;
    const uint64_t c = (uint64_t)(ah ? ah : al) * (uint64_t)(ah ? bl : bh);
    const uint32_t both = (uint32_t)(ah != 0) & (uint32_t)(bh != 0);
    const uint32_t extra = both ? al * bh : 0u;           // the second cross term, low half
    const uint64_t mid = (ll >> 32) + (uint32_t)c;
    ovf |= both | (uint32_t)((c >> 32) != 0) | (uint32_t)(mid >> 32);
    const uint64_t lo = ll + ((uint64_t)((uint32_t)c + extra) << 32);
    const uint64_t s = acc + lo;
    ovf |= (uint32_t)(s < lo);
    return s;
}

// acc + a*b for b < 2^32 (a neighbour count: steps whose passive child is a
// single vertex), with the same overflow rule, from two 32-bit products:
// a*b = (ah*b)*2^32 + al*b reaches 2^64 exactly when ah*b >= 2^32 or
// lo32(ah*b) + hi32(al*b) >= 2^32.
__host__ __device__ __forceinline__ uint64_t mad_ovf_n32(uint64_t acc, uint64_t a, uint32_t b, uint32_t &ovf) {
    const uint64_t ll = (uint64_t)(uint32_t)a * b;
    const uint64_t c = (a >> 32) * (uint64_t)b;
    const uint64_t mid = (ll >> 32) + (uint32_t)c;
    ovf |= (uint32_t)((c >> 32) != 0) | (uint32_t)(mid >> 32);
    const uint64_t lo = ll + (c << 32);
    const uint64_t s = acc + lo;
    ovf |= (uint32_t)(s < lo);
    return s;
}

// ---------------------------------------------------------- residues mod p

// An odd modulus p = 2^w - c below 2^63 (61 <= w <= 63, c <= 2^16; a prime
// when the residues feed the Chinese remainder theorem); wrap = 2^64 mod p.  The DP commutes with
// reduction modulo p (it uses only + and *), so running it on residues gives
// X mod p; with X mod 2^64 the residues determine X below their product.
struct Modulus {
    uint64_t p, c, wrap;
    int w;
};

// x mod p for any x < 2^128, by folding x = hi * 2^w + lo into hi * c + lo.
__host__ __device__ __forceinline__ uint64_t mod_fold(unsigned __int128 x, const Modulus &m) {
    const uint64_t mask = (1ull << m.w) - 1;
    x = (x >> m.w) * m.c + (uint64_t)(x & mask);        // < 2^(128-w) * c + 2^w
    x = (x >> m.w) * m.c + (uint64_t)(x & mask);        // < 2^w + small
    uint64_t r = (uint64_t)((x >> m.w) * m.c + (uint64_t)(x & mask));
    if (r >= m.p) r -= m.p;
    if (r >= m.p) r -= m.p;
    return r;
}

// a + b mod p for a, b < p (< 2^63, so the sum does not wrap).
__host__ __device__ __forceinline__ uint64_t mod_add(uint64_t a, uint64_t b, const Modulus &m) {
    const uint64_t s = a + b;
    return s >= m.p ? s - m.p : s;
}

// acc + a*b mod p for acc, a, b < p.
__host__ __device__ __forceinline__ uint64_t mod_mad(uint64_t acc, uint64_t a, uint64_t b,
                                                     const Modulus &m) {
    return mod_fold((unsigned __int128)a * b + acc, m);
}

// Lazy sums of products: (top * 2^128 + lo) mod p.  A sum of products of
// residues (each below 2^126) is kept exactly as a 128-bit word plus a count
// of its carries, and reduced once.  2^128 mod p = wrap^2 (wrap = 2^(64-w) c
// < 2^19, so wrap^2 < p).
__host__ __device__ __forceinline__ void wide_add_product(unsigned __int128 &lo, uint64_t &top, uint64_t a,
                                                          uint64_t b) {
    const unsigned __int128 pr = (unsigned __int128)a * b;
    lo += pr;
    top += (uint64_t)(lo < pr);
}

// The same for b < 2^32, from two 32-bit products.
__host__ __device__ __forceinline__ void wide_add_product_n32(unsigned __int128 &lo, uint64_t &top, uint64_t a,
                                                              uint32_t b) {
    const unsigned __int128 pr =
        ((unsigned __int128)((a >> 32) * (uint64_t)b) << 32) + (uint64_t)(uint32_t)a * b;
    lo += pr;
    top += (uint64_t)(lo < pr);
}

__host__ __device__ __forceinline__ uint64_t mod_wide_fold(unsigned __int128 lo, uint64_t top,
                                                           const Modulus &m) {
    return mod_fold((unsigned __int128)top * (m.wrap * m.wrap) + mod_fold(lo, m), m);
}

}  // namespace kern
}  // namespace sc
