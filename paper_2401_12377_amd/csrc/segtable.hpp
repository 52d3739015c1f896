// Host-side dependency checks against many kernels at once (step a3).
//
// Up to 64 kernels are held, one per column, each column keeping its
// kernel's (at most eight) ranges side by side: a 64-byte row of starts and
// one of ends, with the number of ranges and a bit mask of the writes.  A
// column is replaced with two vector stores, so the table stays warm in the
// caches when the submitting thread's other work (descriptors, the ring,
// the application's own state) passes through them between two kernels.
// Before any range is compared, one pass over the columns' bounding
// intervals (the smallest start and largest end of each kernel's ranges, 8
// or 4 kernels per vector compare) drops the kernels whose ranges all lie
// apart from the newer kernel's: independent task graphs in disjoint memory
// then cost one compare per 8 held kernels.  Each remaining column is tested
// with one vector compare per range of the newer kernel against all of that
// column's ranges: a newer write meets any range, a newer read meets writes
// only (Algorithm 1 applied both ways, Section III-C).  Bounds are stored
// with the sign bit flipped so that signed compares order them as unsigned
// addresses; unused positions hold [0, 0), which meets nothing.  The table
// asks for no more than 8-byte alignment and the vector loads and stores
// are unaligned ones.
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
    static_assert(ACS_K_MAX == 8, "a column's ranges fill one 64-byte row");

    int64_t s[kCols][ACS_K_MAX];                   // column i: starts of its ranges
    int64_t e[kCols][ACS_K_MAX];                   // column i: ends of its ranges
    int64_t bs[kCols], be[kCols];                  // column i: bounding interval of its ranges
    uint8_t cn[kCols];                             // column i: ranges held
    uint8_t wb[kCols];                             // column i: bit m set when range m is a write

    SegTable()
    {
        for (int i = 0; i < kCols; i++) {
            for (int m = 0; m < ACS_K_MAX; m++) s[i][m] = e[i][m] = kEmpty;
            bs[i] = be[i] = kEmpty;
            cn[i] = wb[i] = 0;
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

    // Column i takes the ranges of d (replacing what it held).
    void put(int i, const Desc &d)
    {
#if defined(__x86_64__)
        static const bool v512 = __builtin_cpu_supports("avx512f");
        if (v512) {
            put_avx512(i, d);
            return;
        }
#endif
        const uint32_t n = d.nseg < (uint32_t)ACS_K_MAX ? d.nseg : (uint32_t)ACS_K_MAX;
        int64_t ss[ACS_K_MAX], ee[ACS_K_MAX];
        for (uint32_t m = 0; m < (uint32_t)ACS_K_MAX; m++) {
            ss[m] = m < n ? (int64_t)(d.s[m] ^ 0x8000000000000000ull) : kEmpty;
            ee[m] = m < n ? (int64_t)(d.e[m] ^ 0x8000000000000000ull) : kEmpty;
        }
        memcpy(s[i], ss, sizeof(ss));
        memcpy(e[i], ee, sizeof(ee));
        cn[i] = (uint8_t)n;
        wb[i] = (uint8_t)(d.wbits & ((1u << n) - 1u));
        bounds(d, bs[i], be[i]);
    }

    // Segment pairs the definition compares for d against the columns `cols`.
    uint64_t pair_tests(uint64_t cols, const Desc &d) const
    {
        const uint32_t nw = (uint32_t)__builtin_popcount(d.wbits & ((1u << d.nseg) - 1u)), nr = d.nseg - nw;
        uint64_t all = 0, wr = 0;
        for (uint64_t c = cols; c; c &= c - 1) {
            const int i = __builtin_ctzll(c);
            all += cn[i];
            wr += (uint64_t)__builtin_popcount(wb[i]);
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
        for (uint64_t c = cols; c; c &= c - 1) {
            const int i = __builtin_ctzll(c);
            bool hit = false;
            for (uint32_t a = 0; a < d.nseg && a < (uint32_t)ACS_K_MAX && !hit; a++) {
                const int64_t sa = (int64_t)(d.s[a] ^ 0x8000000000000000ull), ea = (int64_t)(d.e[a] ^ 0x8000000000000000ull);
                const uint32_t pos = ((d.wbits >> a) & 1u) ? ((1u << cn[i]) - 1u) : wb[i];
                for (int m = 0; m < ACS_K_MAX; m++)
                    if (((pos >> m) & 1u) && e[i][m] > sa && ea > s[i][m]) hit = true;
            }
            if (hit) out |= 1ull << i;
        }
        return out;
    }

#if defined(__x86_64__)
    __attribute__((target("avx512f"))) void put_avx512(int i, const Desc &d)
    {
        const uint32_t n = d.nseg < (uint32_t)ACS_K_MAX ? d.nseg : (uint32_t)ACS_K_MAX;
        const __mmask8 k = (__mmask8)((1u << n) - 1u);
        const __m512i flip = _mm512_set1_epi64((long long)0x8000000000000000ull), empty = _mm512_set1_epi64(kEmpty);
        const __m512i sv = _mm512_mask_xor_epi64(empty, k, _mm512_loadu_si512(d.s), flip);
        const __m512i ev = _mm512_mask_xor_epi64(empty, k, _mm512_loadu_si512(d.e), flip);
        _mm512_storeu_si512(s[i], sv);
        _mm512_storeu_si512(e[i], ev);
        cn[i] = (uint8_t)n;
        wb[i] = (uint8_t)(d.wbits & k);
        // bounding interval: smallest start and largest end over the used positions
        bs[i] = n ? _mm512_mask_reduce_min_epi64(k, sv) : kEmpty;
        be[i] = n ? _mm512_mask_reduce_max_epi64(k, ev) : kEmpty;
    }

    // one column's starts and ends in one register each; a range of d against
    // all of them in two compares
    __attribute__((target("avx512f"))) uint64_t conflicts_avx512(uint64_t cols, const Desc &d) const
    {
        const uint32_t na = d.nseg < (uint32_t)ACS_K_MAX ? d.nseg : (uint32_t)ACS_K_MAX;
        __m512i sa[ACS_K_MAX], ea[ACS_K_MAX];
        for (uint32_t a = 0; a < na; a++) {
            sa[a] = _mm512_set1_epi64((long long)(d.s[a] ^ 0x8000000000000000ull));
            ea[a] = _mm512_set1_epi64((long long)(d.e[a] ^ 0x8000000000000000ull));
        }
        uint64_t out = 0;
        for (uint64_t c = cols; c; c &= c - 1) {
            const int i = __builtin_ctzll(c);
            const __m512i sv = _mm512_loadu_si512(s[i]), ev = _mm512_loadu_si512(e[i]);
            const __mmask8 used = (__mmask8)((1u << cn[i]) - 1u), wr = (__mmask8)wb[i];
            for (uint32_t a = 0; a < na; a++) {
                const __mmask8 k = ((d.wbits >> a) & 1u) ? used : wr;
                if (_mm512_mask_cmpgt_epi64_mask(_mm512_mask_cmpgt_epi64_mask(k, ev, sa[a]), ea[a], sv)) {
                    out |= 1ull << i;
                    break;
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

    // the same with two 4-wide halves per column
    __attribute__((target("avx2"))) uint64_t conflicts_avx2(uint64_t cols, const Desc &d) const
    {
        const uint32_t na = d.nseg < (uint32_t)ACS_K_MAX ? d.nseg : (uint32_t)ACS_K_MAX;
        uint64_t out = 0;
        for (uint64_t c = cols; c; c &= c - 1) {
            const int i = __builtin_ctzll(c);
            const __m256i s0 = _mm256_loadu_si256((const __m256i *)&s[i][0]), s1 = _mm256_loadu_si256((const __m256i *)&s[i][4]);
            const __m256i e0 = _mm256_loadu_si256((const __m256i *)&e[i][0]), e1 = _mm256_loadu_si256((const __m256i *)&e[i][4]);
            const uint32_t used = (1u << cn[i]) - 1u, wr = wb[i];
            for (uint32_t a = 0; a < na; a++) {
                const __m256i sa = _mm256_set1_epi64x((long long)(d.s[a] ^ 0x8000000000000000ull));
                const __m256i ea = _mm256_set1_epi64x((long long)(d.e[a] ^ 0x8000000000000000ull));
                const uint32_t k = ((d.wbits >> a) & 1u) ? used : wr;
                const uint32_t lo4 = (uint32_t)_mm256_movemask_pd(
                    _mm256_castsi256_pd(_mm256_and_si256(_mm256_cmpgt_epi64(e0, sa), _mm256_cmpgt_epi64(ea, s0))));
                const uint32_t hi4 = (uint32_t)_mm256_movemask_pd(
                    _mm256_castsi256_pd(_mm256_and_si256(_mm256_cmpgt_epi64(e1, sa), _mm256_cmpgt_epi64(ea, s1))));
                if ((lo4 | (hi4 << 4)) & k) {
                    out |= 1ull << i;
                    break;
                }
            }
        }
        return out;
    }
#endif
};

}  // namespace acs
