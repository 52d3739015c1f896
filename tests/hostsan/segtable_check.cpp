// Checks the host's vectorised dependency test (segtable.hpp) against the
// pairwise definition (descs_conflict) on random kernels: every instruction
// set the host offers, tables placed at misaligned addresses, segment counts
// 1-8 with random write masks, ranges that touch, nest, or stand apart.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <random>

#include "segtable.hpp"

using namespace acs;

static Desc random_desc(std::mt19937_64 &r)
{
    Desc d;
    d.nseg = 1 + (uint32_t)(r() % ACS_K_MAX);
    const uint32_t nw = (uint32_t)(r() % (d.nseg + 1));
    d.wbits = (1u << nw) - 1u;   // writes first, as make_desc orders them
    for (uint32_t k = 0; k < d.nseg; k++) {
        const int kind = (int)(r() % 8);
        uint64_t s, e;
        if (kind == 0) {
            s = 0;
            e = UINT64_MAX;   // all memory
        } else if (kind == 1) {
            s = UINT64_MAX - 64 - (r() % 64);
            e = s + 1 + (r() % 64);
        } else {
            s = (r() % 4096) * 16;   // small space: frequent overlaps and touching ends
            e = s + 1 + (r() % 512);
        }
        d.s[k] = s;
        d.e[k] = e;
    }
    return d;
}

int main(int argc, char **argv)
{
    const int rounds = argc > 1 ? atoi(argv[1]) : 20000;
    std::mt19937_64 r(7);
    // tables at 8-byte offsets from a 64-byte boundary
    alignas(64) static unsigned char buf[8 * sizeof(SegTable) + 64];
    long checked = 0, hits = 0;
    for (int off = 0; off < 8; off++) {
        SegTable *t = new (buf + 8 * off + off * sizeof(SegTable)) SegTable();
        Desc held[64];
        for (int i = 0; i < 64; i++) {
            held[i] = random_desc(r);
            t->put(i, held[i]);
        }
        for (int it = 0; it < rounds / 8; it++) {
            const Desc nd = random_desc(r);
            const uint64_t cols = r() & r();
            uint64_t want = 0, tests = 0;
            for (int i = 0; i < 64; i++)
                if ((cols >> i) & 1u) {
                    uint64_t tt = 0;
                    if (descs_conflict(held[i], nd, &tt)) want |= 1ull << i;
                    tests += tt;
                }
            const uint64_t got[3] = {t->conflicts_scalar(cols, nd), t->conflicts(cols, nd),
#if defined(__x86_64__)
                                     __builtin_cpu_supports("avx2") ? t->conflicts_avx2(cols, nd) : want
#else
                                     want
#endif
            };
            for (int v = 0; v < 3; v++)
                if (got[v] != want) {
                    printf("MISMATCH variant %d offset %d round %d: %llx vs %llx\n", v, off, it,
                           (unsigned long long)got[v], (unsigned long long)want);
                    return 1;
                }
            if (t->pair_tests(cols, nd) != tests) {
                printf("TEST COUNT MISMATCH offset %d round %d\n", off, it);
                return 1;
            }
            // replace a random column, as the window and the host list do
            const int c = (int)(r() % 64);
            held[c] = random_desc(r);
            t->put(c, held[c]);
            checked++;
            hits += __builtin_popcountll(want);
        }
        t->~SegTable();
    }
    printf("ok %ld checks, %ld conflicts\n", checked, hits);
    return 0;
}
