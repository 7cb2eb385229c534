"""The device's exact arithmetic (csrc/exact.h), compiled for the host with
g++, against unsigned 128-bit arithmetic: both uint64 multiply-adds (residue
and overflow flag) on edge values around every 32-bit and 64-bit boundary and
on random pairs, and the residue operations modulo the three primes."""
import os
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1903_04395_amd", "csrc", "exact.h")

HARNESS = textwrap.dedent(r"""
    #include <cstdio>
    #include <random>
    #include "exact.h"
    typedef unsigned __int128 u128;
    static int check(uint64_t acc, uint64_t a, uint64_t b) {
        uint32_t ovf = 0, ovf3 = 0;
        uint64_t got = sc::kern::mad_ovf(acc, a, b, ovf);
        uint64_t got3 = sc::kern::mad_ovf3(acc, a, b, ovf3);
        u128 p = (u128)a * b, s = (u128)acc + (uint64_t)p;
        uint64_t want = (uint64_t)s;
        int want_ovf = (p >> 64) != 0 || (s >> 64) != 0;
        if (got != want || (ovf != 0) != want_ovf || got3 != want || (ovf3 != 0) != want_ovf) {
            printf("FAIL %llu %llu %llu\n", (unsigned long long)acc, (unsigned long long)a, (unsigned long long)b);
            return 1;
        }
        return 0;
    }
    int main() {
        const uint64_t edge[] = {0, 1, 2, 3, 0xffffffffull, 0x100000000ull, 0x100000001ull,
                                 0x1ffffffffull, 0xfffffffeull, 0x80000000ull, 0x7fffffffffffffffull,
                                 0x8000000000000000ull, 0xffffffffffffffffull, 0xfffffffffffffffeull,
                                 0x0000000100000000ull, 0x00000000ffffffffull, 4294967296ull * 3 + 7,
                                 0x123456789abcdefull, 0xfedcba9876543210ull};
        int bad = 0;
        long n = 0;
        for (uint64_t a : edge) for (uint64_t b : edge) for (uint64_t c : edge) { bad += check(c, a, b); ++n; }
        std::mt19937_64 g(12345);
        for (long i = 0; i < 2000000; ++i) {
            uint64_t a = g(), b = g(), c = g();
            int m = i % 8;                       // vary magnitudes: 0..64-bit operands
            a >>= (g() % 64) * (m & 1);
            b >>= (g() % 64) * ((m >> 1) & 1);
            c >>= (g() % 64) * ((m >> 2) & 1);
            bad += check(c, a, b);
            ++n;
        }
        // products just below and at 2^64
        for (uint64_t a = 1; a < 200000; a += 7) {
            uint64_t b = ~0ull / a;
            bad += check(0, a, b) + check(0, a, b + 1) + check(~0ull - a * b, a, b) + check(~0ull - a * b + 1, a, b);
            n += 4;
        }
        // second operand below 2^32 (neighbour counts)
        for (long i = 0; i < 2000000; ++i) {
            uint64_t a = g(), c = g();
            uint32_t b = (uint32_t)g();
            const int m = i % 8;
            a >>= (g() % 64) * (m & 1);
            b >>= (g() % 32) * ((m >> 1) & 1);
            c >>= (g() % 64) * ((m >> 2) & 1);
            if (i % 97 == 0) { a = ~0ull / (b ? b : 1); c = ~0ull - a * b + (g() & 1); }
            uint32_t o1 = 0, o2 = 0;
            const uint64_t r1 = sc::kern::mad_ovf_n32(c, a, b, o1);
            const uint64_t r2 = sc::kern::mad_ovf(c, a, b, o2);
            if (r1 != r2 || o1 != o2) { printf("FAIL n32 %llu %u %llu\n", (unsigned long long)a, b, (unsigned long long)c); bad++; }
            u128 lo1 = ((u128)g() << 64) | g(), lo2 = lo1;
            uint64_t t1 = g() >> 8, t2 = t1;
            sc::kern::wide_add_product_n32(lo1, t1, a, b);
            sc::kern::wide_add_product(lo2, t2, a, b);
            if (lo1 != lo2 || t1 != t2) { printf("FAIL wide n32\n"); bad++; }
            n += 2;
        }
        // residues modulo the primes 2^61 - 1, 2^62 - 57, 2^63 - 25
        const sc::kern::Modulus mods[3] = {{(1ull << 61) - 1, 1, 8, 61},
                                           {(1ull << 62) - 57, 57, 228, 62},
                                           {(1ull << 63) - 25, 25, 50, 63}};
        for (const auto &md : mods) {
            if (((u128)1 << 64) % md.p != md.wrap) { printf("BAD wrap\n"); return 1; }
            std::mt19937_64 h(md.p);
            for (long i = 0; i < 1000000; ++i) {
                u128 x = ((u128)h() << 64) | h();
                if (i % 3 == 0) x >>= (h() % 128);
                if (sc::kern::mod_fold(x, md) != (uint64_t)(x % md.p)) { printf("FAIL fold\n"); bad++; }
                uint64_t a = h() % md.p, b = h() % md.p, c = h() % md.p;
                if (i % 5 == 0) { a = md.p - 1 - (h() % 3); b = md.p - 1 - (h() % 3); c = md.p - 1; }
                if (sc::kern::mod_add(a, b, md) != (uint64_t)(((u128)a + b) % md.p)) { printf("FAIL add\n"); bad++; }
                if (sc::kern::mod_mad(c, a, b, md) != (uint64_t)(((u128)a * b + c) % md.p)) { printf("FAIL mad\n"); bad++; }
                n += 3;
            }
            // lazy sums of up to 40 products of residues against term-by-term reduction
            const uint64_t w2 = (uint64_t)((((u128)1 << 64) % md.p) * (((u128)1 << 64) % md.p) % md.p);
            for (long i = 0; i < 200000; ++i) {
                u128 lo = 0;
                uint64_t top = 0, want = 0;
                const int terms = 1 + (int)(h() % 40);
                for (int j = 0; j < terms; ++j) {
                    uint64_t a = h() % md.p, b = h() % md.p;
                    if (i % 4 == 0) { a = md.p - 1; b = md.p - 1 - (h() % 2); }
                    sc::kern::wide_add_product(lo, top, a, b);
                    want = (uint64_t)(((u128)a * b % md.p + want) % md.p);
                }
                if (sc::kern::mod_wide_fold(lo, top, md) != want) { printf("FAIL wide\n"); bad++; }
                // arbitrary (top, lo), against (top * (2^128 mod p) + lo) mod p
                const u128 x = ((u128)h() << 64) | h();
                const uint64_t t2 = h() >> (h() % 64);
                const uint64_t ref = (uint64_t)(((u128)(t2 % md.p) * w2 % md.p + x % md.p) % md.p);
                if (sc::kern::mod_wide_fold(x, t2, md) != ref) { printf("FAIL widefold\n"); bad++; }
                n += 2;
            }
        }
        printf("%s %ld\n", bad ? "BAD" : "OK", n);
        return bad != 0;
    }
""")


def test_mad_ovf_matches_128bit(tmp_path):
    src = tmp_path / "h.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "h"
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__host__=", "-D__device__=", "-D__forceinline__=inline",
                    "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("OK"), out.stdout[-500:]
