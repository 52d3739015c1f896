// Host-side internals of libacs (not part of the public ABI).
#pragma once
#include <stdint.h>

#include <memory>
#if defined(__x86_64__)
#include <immintrin.h>
#endif
#include <string>
#include <vector>

#include "acs.h"
#include "acs_tasks.h"

namespace acs {

// A submitted kernel after its segment lists were normalised (step a1).
// Segments are [s, e) byte ranges, reads first then writes; bit k of wbits
// marks segment k as a write.  Unused entries are [0, 0).
struct Desc {
    uint64_t seq = 0;
    int32_t kid = 0;
    uint32_t npieces = 1;
    uint32_t nseg = 0;
    uint32_t wbits = 0;
    uint64_t s[ACS_K_MAX] = {};
    uint64_t e[ACS_K_MAX] = {};
    alignas(8) uint8_t args[ACS_ARGS_MAX] = {};
    uint32_t args_size = 0;
};

// Overlap of two half-open ranges (Algorithm 1's test).
inline bool ranges_overlap(uint64_t s1, uint64_t e1, uint64_t s2, uint64_t e2) { return s1 < e2 && e1 > s2; }

#if defined(__x86_64__)
// The same test with four positions per AVX2 compare: every position of the
// older kernel at once (unused positions hold [0, 0), which meets nothing),
// unsigned order by flipping the sign bits.
__attribute__((target("avx2"))) inline bool descs_conflict_avx2(const Desc &older, const Desc &newer)
{
    const __m256i sign = _mm256_set1_epi64x((long long)0x8000000000000000ull);
    const __m256i os0 = _mm256_xor_si256(_mm256_loadu_si256(reinterpret_cast<const __m256i *>(older.s)), sign);
    const __m256i os1 = _mm256_xor_si256(_mm256_loadu_si256(reinterpret_cast<const __m256i *>(older.s + 4)), sign);
    const __m256i oe0 = _mm256_xor_si256(_mm256_loadu_si256(reinterpret_cast<const __m256i *>(older.e)), sign);
    const __m256i oe1 = _mm256_xor_si256(_mm256_loadu_si256(reinterpret_cast<const __m256i *>(older.e + 4)), sign);
    const uint32_t w = older.wbits;
    auto bitmask = [](uint32_t b) { return (long long)(0ull - (uint64_t)(b & 1u)); };
    const __m256i wm0 = _mm256_set_epi64x(bitmask(w >> 3), bitmask(w >> 2), bitmask(w >> 1), bitmask(w));
    const __m256i wm1 = _mm256_set_epi64x(bitmask(w >> 7), bitmask(w >> 6), bitmask(w >> 5), bitmask(w >> 4));
    for (uint32_t a = 0; a < newer.nseg; a++) {
        const __m256i sa = _mm256_set1_epi64x((long long)(newer.s[a] ^ 0x8000000000000000ull));
        const __m256i ea = _mm256_set1_epi64x((long long)(newer.e[a] ^ 0x8000000000000000ull));
        // newer [sa, ea) meets older [s, e) iff sa < e and ea > s
        __m256i m0 = _mm256_and_si256(_mm256_cmpgt_epi64(oe0, sa), _mm256_cmpgt_epi64(ea, os0));
        __m256i m1 = _mm256_and_si256(_mm256_cmpgt_epi64(oe1, sa), _mm256_cmpgt_epi64(ea, os1));
        if (!((newer.wbits >> a) & 1u)) {   // a read meets only writes
            m0 = _mm256_and_si256(m0, wm0);
            m1 = _mm256_and_si256(m1, wm1);
        }
        const __m256i m = _mm256_or_si256(m0, m1);
        if (!_mm256_testz_si256(m, m)) return true;
    }
    return false;
}
#endif

// Dependency of `newer` on `older`: the newer kernel's writes against all of
// the older one's ranges, and its reads against the older one's writes.
// make_desc lists a kernel's writes first, so the writes of a descriptor are
// its first popcount(wbits) positions; each row of tests is branch-free.
// `tests` counts the segment pairs the definition compares.
inline bool descs_conflict(const Desc &older, const Desc &newer, uint64_t *tests)
{
#if defined(__x86_64__)
    static const bool avx2 = __builtin_cpu_supports("avx2");
    if (avx2) {
        if (tests) {
            const uint32_t nwn = (uint32_t)__builtin_popcount(newer.wbits), nwo = (uint32_t)__builtin_popcount(older.wbits);
            *tests += (uint64_t)nwn * older.nseg + (uint64_t)(newer.nseg - nwn) * nwo;
        }
        return descs_conflict_avx2(older, newer);
    }
#endif
    const uint32_t nn = newer.nseg, no = older.nseg;
    const uint32_t nwn = (uint32_t)__builtin_popcount(newer.wbits), nwo = (uint32_t)__builtin_popcount(older.wbits);
    const bool packed = newer.wbits == (1u << nwn) - 1u && older.wbits == (1u << nwo) - 1u;
    uint64_t n = 0;
    bool hit = false;
    for (uint32_t a = 0; a < nn && !hit; a++) {
        const uint64_t s = newer.s[a], e = newer.e[a];
        // a write meets every range of the older kernel, a read only its writes
        const bool wa = (newer.wbits >> a) & 1u;
        const uint32_t lim = packed ? (wa ? no : nwo) : no;
        bool row = false;
        for (uint32_t b = 0; b < lim; b++) {
            const bool wb = (older.wbits >> b) & 1u;
            row |= (wa | wb) & (s < older.e[b]) & (e > older.s[b]);
        }
        n += lim;
        hit = row;
    }
    if (tests) *tests += n;
    return hit;
}

// Checks and normalises one submission (validation, dropping empty ranges,
// merging ranges beyond ACS_K_MAX, piece count).  Returns ACS_OK or ACS_EINVAL.
int make_desc(int32_t kid, const acs_seg *r, int32_t nr, const acs_seg *w, int32_t nw, const void *args,
              size_t args_size, int32_t wg_per_task, Desc &out, bool *coalesced, std::string *why);

void set_error(int code, const std::string &msg);

// Interface of one execution path behind a window.
class Path {
public:
    virtual ~Path() = default;
    virtual int start() { return ACS_OK; }
    virtual int submit(const Desc &d) = 0;
    // groups are independent windows: only the device path keeps them apart
    virtual int submit_group(const Desc &d, int32_t group) { (void)group; return submit(d); }
    virtual int sync(uint64_t timeout_ns) = 0;                     // 0 = wait forever
    virtual int sync_group(int32_t group, uint64_t timeout_ns) { (void)group; return sync(timeout_ns); }
    virtual int poll() { return ACS_OK; }
    virtual int scheduled_list(acs_entry *out, int32_t cap, int32_t *n) = 0;
    virtual int trace_read(acs_trace_rec *out, int64_t cap, int64_t *n) = 0;
    virtual int take_ready(uint64_t *, int32_t, int32_t *) { return ACS_ESTATE; }
    virtual int complete(uint64_t, int32_t) { return ACS_ESTATE; }
    virtual int shutdown() { return ACS_OK; }
    // drain and release execution resources, keep stats/trace readable
    virtual int stop() { return sync(0); }
    virtual void stats(acs_stats &s) = 0;
};

std::unique_ptr<Path> make_inorder_path(const acs_config &cfg);
std::unique_ptr<Path> make_plain_path(int32_t W, const acs_config &cfg);
std::unique_ptr<Path> make_manual_path(int32_t W, const acs_config &cfg);
std::unique_ptr<Path> make_device_path(int32_t W, const acs_config &cfg);
// The device path without allocation (acs_window_configure_noalloc): null
// with *rc set when the device's static state is taken or out of range.
std::unique_ptr<Path> make_device_path_static(int32_t W, const acs_config &cfg, void *host, uint64_t host_bytes,
                                              void *stream, int *rc);
std::unique_ptr<Path> make_events_path(const acs_config &cfg);

uint64_t now_ns();

}  // namespace acs

// The window object behind the opaque acs_window handle.
struct acs_window {
    int32_t W = 0;
    acs_config cfg;
    bool configured = false;
    bool started = false;
    bool stopped = false;
    uint64_t next_seq = 0;
    uint64_t coalesced = 0;
    std::unique_ptr<acs::Path> path;
    bool recording = false;              // between acs_graph_begin and acs_graph_end
    std::vector<acs::Desc> recorded;
};
