// Checks the host's vectorised dependency test (segtable.hpp) against the
// pairwise definition (descs_conflict) on random kernels: every instruction
// set the host offers, tables placed at misaligned addresses, segment counts
// 1-8 with random write masks, ranges that touch, nest, or stand apart, and
// kernels kept inside one of a few far-apart blocks of memory (so that the
// bounding-interval filter drops columns) or spread over several of them.
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
    // half of the kernels keep to one block out of 8, 1 GiB apart
    const bool block = r() % 2;
    const uint64_t base = (r() % 8) << 30;
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
            // small space: frequent overlaps and touching ends; each range in
            // a block of its own when the kernel is not kept to one
            s = (block ? base : (r() % 8) << 30) + (r() % 4096) * 16;
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
    long checked = 0, hits = 0, filtered = 0;
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
            int64_t lo, hi;
            SegTable::bounds(nd, lo, hi);
            const uint64_t ns = t->near_scalar(cols, lo, hi);
            if ((want & ~ns) != 0 || (ns & ~cols) != 0) {
                printf("FILTER DROPPED A CONFLICT offset %d round %d\n", off, it);
                return 1;
            }
            filtered += __builtin_popcountll(cols & ~ns);
            const uint64_t got[6] = {t->conflicts_scalar(cols, nd), t->conflicts(cols, nd), t->conflicts_scalar(ns, nd),
#if defined(__x86_64__)
                                     __builtin_cpu_supports("avx2") ? t->conflicts_avx2(cols, nd) : want,
                                     __builtin_cpu_supports("avx2") ? t->conflicts_avx2(t->near_avx2(cols, lo, hi), nd) : want,
                                     __builtin_cpu_supports("avx512f") ? (t->near_avx512(cols, lo, hi) == ns ? want : ~want) : want
#else
                                     want, want, want
#endif
            };
            for (int v = 0; v < 6; v++)
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
    printf("ok %ld checks, %ld conflicts, %ld columns dropped by the bounds\n", checked, hits, filtered);
    return 0;
}
