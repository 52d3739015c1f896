// Host-side dependency checks against many kernels at once (step a3).
//
// The ranges of up to 64 kernels are held by position: row m of the table
// holds the m-th range of every kernel (column i is kernel i), with bit masks
// of the columns whose m-th range exists and of those where it is a write.
// A newer kernel's write is compared with every held range, its read only
// with held writes (the masks pick the columns), and one vector compare
// tests one range of the newer kernel against the same position of 8
// (AVX-512) or 4 (AVX2) held kernels.  Columns already found in conflict
// are not tested again.  Before any of that, one pass over the columns'
// bounding intervals (the smallest start and largest end of each kernel's
// ranges) drops the kernels whose ranges all lie apart from the newer
// kernel's: independent task graphs in disjoint memory then cost one
// compare per 8 held kernels.  Bounds are stored with the sign bit flipped so that
// signed compares order them as unsigned addresses; empty positions hold
// [0, 0), which meets nothing.  The table asks for no more than 8-byte
// alignment and the vector loads are unaligned ones.  The relation is that
// of Algorithm 1 applied both ways (Section III-C): a newer write meets any
// range, a newer read meets writes only.
#pragma once
#include <stdint.h>
#include <string.h>

#if defined(__x86_64__)
#include <immintrin.h>
#endif

#include "internal.hpp"

namespace acs {

struct SegTable {
    static constexpr int kCols = 64;
    static constexpr int64_t kEmpty = INT64_MIN;   // flipped 0

    int64_t s[ACS_K_MAX][kCols];
    int64_t e[ACS_K_MAX][kCols];
    uint64_t used[ACS_K_MAX];                      // bit i of row m: kernel i has an m-th range
    uint64_t wrow[ACS_K_MAX];                      // bit i of row m: that range is a write
    int64_t bs[kCols], be[kCols];                  // column i: bounding interval of its ranges
    uint8_t cn[kCols];                             // column i: ranges held (rows at and past it are empty)

    SegTable()
    {
        for (int m = 0; m < ACS_K_MAX; m++) {
            for (int i = 0; i < kCols; i++) s[m][i] = e[m][i] = kEmpty;
            used[m] = wrow[m] = 0;
        }
        for (int i = 0; i < kCols; i++) {
            bs[i] = be[i] = kEmpty;
            cn[i] = 0;
        }
    }

    // Bounding interval of d's ranges, flipped; [0, 0) when it has none.
    static void bounds(const Desc &d, int64_t &lo, int64_t &hi)
    {
        lo = hi = kEmpty;
        for (uint32_t m = 0; m < d.nseg && m < (uint32_t)ACS_K_MAX; m++) {
            const int64_t a = (int64_t)(d.s[m] ^ 0x8000000000000000ull), b = (int64_t)(d.e[m] ^ 0x8000000000000000ull);
            lo = m == 0 || a < lo ? a : lo;
            hi = m == 0 || b > hi ? b : hi;
        }
    }

    // Column i takes the ranges of d (replacing what it held).  Rows at and
    // past both the old and the new range count are empty already.
    void put(int i, const Desc &d)
    {
        const uint64_t bit = 1ull << i;
        const uint32_t n = d.nseg < (uint32_t)ACS_K_MAX ? d.nseg : (uint32_t)ACS_K_MAX;
        const uint32_t rows = n > cn[i] ? n : cn[i];
        for (uint32_t m = 0; m < rows; m++) {
            const bool u = m < n, w = u && ((d.wbits >> m) & 1u);
            s[m][i] = u ? (int64_t)(d.s[m] ^ 0x8000000000000000ull) : kEmpty;
            e[m][i] = u ? (int64_t)(d.e[m] ^ 0x8000000000000000ull) : kEmpty;
            used[m] = u ? (used[m] | bit) : (used[m] & ~bit);
            wrow[m] = w ? (wrow[m] | bit) : (wrow[m] & ~bit);
        }
        cn[i] = (uint8_t)n;
        bounds(d, bs[i], be[i]);
    }

    // Segment pairs the definition compares for d against the columns `cols`.
    uint64_t pair_tests(uint64_t cols, const Desc &d) const
    {
        const uint32_t nw = (uint32_t)__builtin_popcount(d.wbits & ((1u << d.nseg) - 1u)), nr = d.nseg - nw;
        uint64_t all = 0, wr = 0;
        for (int m = 0; m < ACS_K_MAX; m++) {
            all += (uint64_t)__builtin_popcountll(used[m] & cols);
            wr += (uint64_t)__builtin_popcountll(wrow[m] & cols);
        }
        return nw * all + nr * wr;
    }

    // Bit i of the result: d depends on the kernel of column i (i in cols).
    uint64_t conflicts(uint64_t cols, const Desc &d) const
    {
        int64_t lo, hi;
        bounds(d, lo, hi);
#if defined(__x86_64__)
        static const int isa = __builtin_cpu_supports("avx512f") ? 2 : (__builtin_cpu_supports("avx2") ? 1 : 0);
        if (isa == 2) {
            const uint64_t c = near_avx512(cols, lo, hi);
            return c ? conflicts_avx512(c, d) : 0;
        }
        if (isa == 1) {
            const uint64_t c = near_avx2(cols, lo, hi);
            return c ? conflicts_avx2(c, d) : 0;
        }
#endif
        const uint64_t c = near_scalar(cols, lo, hi);
        return c ? conflicts_scalar(c, d) : 0;
    }

    // The columns of `cols` whose bounding interval meets [lo, hi) (flipped
    // bounds): a superset of the columns any range of [lo, hi) can meet.
    uint64_t near_scalar(uint64_t cols, int64_t lo, int64_t hi) const
    {
        uint64_t out = 0;
        for (uint64_t c = cols; c; c &= c - 1) {
            const int i = __builtin_ctzll(c);
            if (be[i] > lo && hi > bs[i]) out |= 1ull << i;
        }
        return out;
    }

    uint64_t conflicts_scalar(uint64_t cols, const Desc &d) const
    {
        uint64_t out = 0;
        for (uint32_t a = 0; a < d.nseg && a < (uint32_t)ACS_K_MAX; a++) {
            const int64_t sa = (int64_t)(d.s[a] ^ 0x8000000000000000ull), ea = (int64_t)(d.e[a] ^ 0x8000000000000000ull);
            const bool wa = (d.wbits >> a) & 1u;
            for (int m = 0; m < ACS_K_MAX; m++) {
                uint64_t c = cols & (wa ? used[m] : wrow[m]) & ~out;
                for (; c; c &= c - 1) {
                    const int i = __builtin_ctzll(c);
                    if (e[m][i] > sa && ea > s[m][i]) out |= 1ull << i;
                }
            }
        }
        return out;
    }

#if defined(__x86_64__)
    __attribute__((target("avx512f"))) uint64_t conflicts_avx512(uint64_t cols, const Desc &d) const
    {
        uint64_t out = 0;
        for (uint32_t a = 0; a < d.nseg && a < (uint32_t)ACS_K_MAX; a++) {
            const __m512i sa = _mm512_set1_epi64((long long)(d.s[a] ^ 0x8000000000000000ull));
            const __m512i ea = _mm512_set1_epi64((long long)(d.e[a] ^ 0x8000000000000000ull));
            const bool wa = (d.wbits >> a) & 1u;
            for (int m = 0; m < ACS_K_MAX; m++) {
                // columns still undecided that hold a range this position can meet
                const uint64_t c = cols & (wa ? used[m] : wrow[m]) & ~out;
                if (!c) continue;
                for (int g = 0; g < kCols / 8; g++) {
                    const __mmask8 k = (__mmask8)(c >> (8 * g));
                    if (!k) continue;
                    const __m512i sv = _mm512_loadu_si512(&s[m][8 * g]), ev = _mm512_loadu_si512(&e[m][8 * g]);
                    const __mmask8 h = _mm512_mask_cmpgt_epi64_mask(_mm512_mask_cmpgt_epi64_mask(k, ev, sa), ea, sv);
                    out |= (uint64_t)h << (8 * g);
                }
            }
        }
        return out;
    }

    __attribute__((target("avx512f"))) uint64_t near_avx512(uint64_t cols, int64_t lo, int64_t hi) const
    {
        const __m512i l = _mm512_set1_epi64((long long)lo), h = _mm512_set1_epi64((long long)hi);
        uint64_t out = 0;
        for (int g = 0; g < kCols / 8; g++) {
            const __mmask8 k = (__mmask8)(cols >> (8 * g));
            if (!k) continue;
            const __m512i sv = _mm512_loadu_si512(&bs[8 * g]), ev = _mm512_loadu_si512(&be[8 * g]);
            out |= (uint64_t)_mm512_mask_cmpgt_epi64_mask(_mm512_mask_cmpgt_epi64_mask(k, ev, l), h, sv) << (8 * g);
        }
        return out;
    }

    __attribute__((target("avx2"))) uint64_t near_avx2(uint64_t cols, int64_t lo, int64_t hi) const
    {
        const __m256i l = _mm256_set1_epi64x((long long)lo), h = _mm256_set1_epi64x((long long)hi);
        uint64_t out = 0;
        for (int g = 0; g < kCols / 4; g++) {
            const uint32_t k = (uint32_t)(cols >> (4 * g)) & 0xFu;
            if (!k) continue;
            const __m256i m = _mm256_and_si256(_mm256_cmpgt_epi64(_mm256_loadu_si256((const __m256i *)&be[4 * g]), l),
                                               _mm256_cmpgt_epi64(h, _mm256_loadu_si256((const __m256i *)&bs[4 * g])));
            out |= (uint64_t)((uint32_t)_mm256_movemask_pd(_mm256_castsi256_pd(m)) & k) << (4 * g);
        }
        return out;
    }

    __attribute__((target("avx2"))) uint64_t conflicts_avx2(uint64_t cols, const Desc &d) const
    {
        uint64_t out = 0;
        for (uint32_t a = 0; a < d.nseg && a < (uint32_t)ACS_K_MAX; a++) {
            const __m256i sa = _mm256_set1_epi64x((long long)(d.s[a] ^ 0x8000000000000000ull));
            const __m256i ea = _mm256_set1_epi64x((long long)(d.e[a] ^ 0x8000000000000000ull));
            const bool wa = (d.wbits >> a) & 1u;
            for (int m = 0; m < ACS_K_MAX; m++) {
                const uint64_t c = cols & (wa ? used[m] : wrow[m]) & ~out;
                if (!c) continue;
                for (int g = 0; g < kCols / 4; g++) {
                    const uint32_t k = (uint32_t)(c >> (4 * g)) & 0xFu;
                    if (!k) continue;
                    const __m256i h =
                        _mm256_and_si256(_mm256_cmpgt_epi64(_mm256_loadu_si256((const __m256i *)&e[m][4 * g]), sa),
                                         _mm256_cmpgt_epi64(ea, _mm256_loadu_si256((const __m256i *)&s[m][4 * g])));
                    const uint32_t hb = (uint32_t)_mm256_movemask_pd(_mm256_castsi256_pd(h)) & k;
                    out |= (uint64_t)hb << (4 * g);
                }
            }
        }
        return out;
    }
#endif
};

}  // namespace acs
