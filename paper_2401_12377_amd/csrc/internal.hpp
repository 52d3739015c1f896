// Host-side internals of libacs (not part of the public ABI).
#pragma once
#include <stdint.h>

#include <memory>
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

// Dependency of `newer` on `older`: the newer kernel's writes against all of
// the older one's ranges, and its reads against the older one's writes.
inline bool descs_conflict(const Desc &older, const Desc &newer, uint64_t *tests)
{
    uint64_t n = 0;
    bool hit = false;
    for (uint32_t a = 0; a < newer.nseg && !hit; a++) {
        const bool wa = (newer.wbits >> a) & 1u;
        for (uint32_t b = 0; b < older.nseg; b++) {
            const bool wb = (older.wbits >> b) & 1u;
            n++;
            if ((wa || wb) && ranges_overlap(newer.s[a], newer.e[a], older.s[b], older.e[b])) {
                hit = true;
                break;
            }
        }
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
