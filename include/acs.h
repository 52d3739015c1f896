/*
 * acs.h - windowed out-of-order kernel scheduler for MI355X (gfx950).
 *
 * The method is ACS (Durvasula et al., "ACS: Concurrent Kernel Execution on
 * Irregular, Input-Dependent Computational Graphs", arXiv 2401.12377).  Each
 * submitted kernel carries the byte ranges it reads and writes (Section III-C,
 * "Determining inter-kernel dependencies"; Section IV-A, the kernel wrapper and
 * its get_addresses function).  Kernels enter a fixed-size scheduling window
 * in submission order (Section III-D, "Mechanism Walkthrough"); on entry each
 * one is tested for overlap against every kernel already in the window
 * (Algorithm 1), which gives its list of upstream kernels and makes it
 * pending, or ready when that list is empty (Section III-C, "Tracking kernel
 * state at runtime").  Ready kernels run concurrently; a completion removes
 * the kernel from the window and from every upstream list (Section IV-B,
 * Algorithm 2; Section IV-C).
 *
 * Paths (acs_config.path):
 *   ACS_PATH_INORDER  every kernel is launched at submit into one HIP stream;
 *                     no window.  The single-stream baseline of Section II.
 *   ACS_PATH_PLAIN    window checks on the host, ready kernels launched into a
 *                     pool of HIP streams (Section IV-B); a kernel whose
 *                     upstream kernels all run in one stream is launched into
 *                     that stream at once; completions seen through HIP events
 *                     recorded when a completion is needed.
 *   ACS_PATH_DEVICE   window held on the GPU by a persistent scheduler kernel:
 *                     one wavefront keeps one window slot per lane, tests the
 *                     overlaps, builds the ready mask with a ballot and
 *                     publishes ready work to resident worker workgroups that
 *                     run the task bodies and signal completion with atomic
 *                     counters.  The software analogue of ACS-HW (Section IV-C):
 *                     no host round trip per kernel.
 *   ACS_PATH_MANUAL   window only, no GPU: the caller takes ready kernels and
 *                     reports their completion (a stand-in executor for tests).
 *   ACS_PATH_EVENTS   no window: the multi-stream baseline of Section III-A.
 *                     Every kernel is launched at submit into one of n_streams
 *                     streams (that of its newest upstream kernel, else the
 *                     next in turn); an upstream kernel in another stream
 *                     becomes a hipStreamWaitEvent on its completion event.
 *                     Upstream kernels are found with the same range test
 *                     against the last 64 kernels, and a kernel leaves that
 *                     list only once its event has fired.  No trace.
 *
 * Conventions.  Functions return ACS_OK (0) or a negative ACS_E* code.  A
 * window is driven by one host thread at a time.  Device buffers named in
 * task arguments are borrowed: the caller owns them and keeps them alive until
 * acs_sync returns.  Segment lists and argument blocks are copied before
 * acs_submit returns.
 */
#ifndef ACS_H
#define ACS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct acs_window acs_window;

/* A byte range [start, start + size) of virtual memory (Section III-C: a start
 * address and a size).  Zero-size ranges are dropped.  The range
 * {0, UINT64_MAX} stands for "may touch any memory", the conservative fallback
 * of Section IV-A for kernels whose accesses cannot be stated. */
typedef struct {
    uint64_t start;
    uint64_t size;
} acs_seg;

#define ACS_SEG_ALL_START 0ull
#define ACS_SEG_ALL_SIZE UINT64_MAX

/* Kernel states in the window (Section III-C; two bits per slot in Section IV-C). */
enum { ACS_PENDING = 0, ACS_READY = 1, ACS_EXECUTING = 2 };

enum {
    ACS_OK = 0,
    ACS_EINVAL = -1,     /* bad argument: W outside [1,64], unknown kernel id, overflowing range ... */
    ACS_ENOMEM = -2,     /* host or device allocation failed */
    ACS_EAGAIN = -3,     /* input FIFO full and the window is non-blocking (or manual and stalled) */
    ACS_EDEVICE = -4,    /* a HIP call failed */
    ACS_ETIMEDOUT = -5,  /* acs_sync_timeout ran out of time */
    ACS_EKERNEL = -6,    /* a kernel failed; its dependents were not run */
    ACS_ESTATE = -7      /* call not valid in this state (e.g. configure after submit) */
};

enum { ACS_PATH_INORDER = 0, ACS_PATH_PLAIN = 1, ACS_PATH_DEVICE = 2, ACS_PATH_MANUAL = 3, ACS_PATH_EVENTS = 4 };

#define ACS_W_MAX 64       /* one window slot per wavefront lane */
#define ACS_K_MAX 8        /* read + write segments kept per kernel */
#define ACS_ARGS_MAX 64    /* bytes of task arguments */
#define ACS_HOST_CHECK_MAX 128 /* longest host check list (host_check_depth) */

typedef struct {
    int32_t path;            /* ACS_PATH_* (default ACS_PATH_DEVICE) */
    int32_t n_streams;       /* plain and events paths: HIP streams in the pool (default 4) */
    int32_t wg_per_task;     /* workgroups per splittable task body (default 1) */
    int32_t n_workers;       /* device path: worker workgroups (0 = one per compute unit) */
    int32_t queue_depth;     /* input FIFO capacity in kernels (default 4096) */
    int32_t nonblocking;     /* 1: acs_submit returns ACS_EAGAIN when the FIFO is full */
    int32_t trace;           /* 1: record a per-kernel trace (see acs_trace_read) */
    int32_t trace_capacity;  /* kernels the trace can hold (default 1 << 16) */
    int32_t device;          /* HIP device ordinal (default 0) */
    int32_t n_groups;        /* independent windows of W slots each (default 1; see acs_submit_group) */
    int32_t host_check_depth;/* device path, one group: 0 (default) = dependency checks in the window
                                wave; M in [1, ACS_HOST_CHECK_MAX] = the host/device split of
                                Section IV-C: the host checks each kernel against the kernels of
                                the M sequence numbers before it (its scheduled list, possibly
                                stale), the device drops upstream kernels that already completed
                                and holds a kernel back while one more than M older is still in
                                the window.  M may exceed W: the list then also covers kernels
                                that left the window or wait for a slot, so that one long
                                kernel holds back only the kernels more than M after it.  Same
                                schedules; other paths ignore it. */
    int32_t window_check;    /* device path, one group, host_check_depth 0: 0 (default) = the
                                same split inside the device: a wave ahead of the window checks
                                each kernel against the 64 submitted before it and the window
                                wave only drops completed upstream kernels (M = 64 above);
                                1 = the window wave makes the checks itself (Algorithm 1 at
                                insert), as it always does with more than one group.  Same
                                schedules either way. */
    int32_t reserved[4];
} acs_config;

/* One entry of the scheduled list (Section IV-C): the kernels currently in the
 * window.  On the device path the list is a snapshot and may be stale. */
typedef struct {
    uint64_t seq;            /* submission index */
    int32_t kernel_id;
    int32_t state;           /* ACS_PENDING / ACS_READY / ACS_EXECUTING */
    uint64_t upstream_mask;  /* window slots this kernel still waits for */
    int32_t slot;
    int32_t reserved;
} acs_entry;

/* One trace record per kernel (all times on one clock, in nanoseconds). */
typedef struct {
    int64_t seq, slot, kernel_id;
    int64_t ev_insert, ev_dispatch, ev_retire;  /* positions in the window's event order */
    uint64_t valid_mask;     /* slots held by older kernels when this kernel was inserted */
    uint64_t up_mask;        /* its upstream slots at insert */
    int64_t t_start, t_end;  /* execution interval, -1 if not recorded */
    int64_t t_dispatch;      /* when the window made it runnable (device path; else -1) */
    int64_t t_retire;        /* when the window saw it complete (device path; else -1) */
} acs_trace_rec;

typedef struct {
    uint64_t submitted, retired, dispatched;
    uint64_t coalesced;      /* kernels whose segment lists were merged to fit ACS_K_MAX */
    uint64_t overlap_tests;  /* segment-pair tests made by the dependency checks */
    uint64_t poisoned;       /* kernels not run because an upstream kernel failed */
    int32_t path, W;
    int32_t n_workers, n_streams;
    uint64_t kernel_ns;      /* device path, after acs_window_stop: duration of the
                                persistent kernel from HIP events on its stream */
} acs_stats;

/* Fills *cfg with the defaults listed above. */
void acs_config_default(acs_config *cfg);

/* New window of W slots, 1 <= W <= 64 (the paper evaluates W = 32 and 16,
 * Section V and Section VI-D).  NULL on error; see acs_last_error(). */
acs_window *acs_window_create(int32_t W);

/* Chooses the path and its resources; valid before the first submit only.
 * Without this call the window uses acs_config_default(). */
int acs_window_configure(acs_window *w, const acs_config *cfg);

/* For callers that cannot allocate memory (code that must not call hipMalloc
 * or hipHostMalloc: tight serving loops, harnesses that forbid allocation):
 * acs_window_configure for the device path that allocates nothing.
 *   cfg         as for acs_window_configure; path must be ACS_PATH_DEVICE and
 *               trace 0 (ACS_EINVAL otherwise).
 *   host_mem    the caller's pinned, coherent, device-mapped host memory (for
 *               example from acs_host_alloc), 64-byte aligned, at least
 *               ACS_NOALLOC_HOST_BYTES(q, G) bytes with q = queue_depth
 *               rounded up to a power of two (at least 16) and G = n_groups
 *               (ACS_EINVAL if shorter).  It holds the input FIFO and the
 *               control words; the caller keeps it alive and untouched until
 *               acs_window_destroy returns.
 *   stream      the caller's hipStream_t on cfg->device, created non-blocking
 *               and used by nothing else until acs_window_stop or
 *               acs_window_destroy returns: the persistent kernel runs in it.
 * The scheduler state lives in a static device array of 1.6 MiB per device,
 * which each device holds until the process ends; it is cleared by a fill
 * kernel on `stream` before the persistent kernel starts.  One such window
 * per device at a time: a second one on the same device, while the first has
 * not been destroyed, gets ACS_ESTATE (two would share that array).
 * acs_stats.kernel_ns stays 0 (no timing events are created).  Everything
 * else behaves as with acs_window_configure. */
#define ACS_NOALLOC_HOST_BYTES(q, G) (4096ull + 256ull * (uint64_t)(q) * (uint64_t)(G))
int acs_window_configure_noalloc(acs_window *w, const acs_config *cfg, void *host_mem, uint64_t host_bytes,
                                 void *stream);

/* Submits one kernel in program order (Section III-D: kernels enter the
 * input FIFO and then the window in submission order; Section IV-A: the
 * kernel wrapper states the ranges its launch arguments touch).
 *   kernel_id   task type from acs_tasks.h (the body the library runs).
 *   read_segs   n_read byte ranges the kernel reads; write_segs likewise.
 *               Beyond ACS_K_MAX segments in total, neighbouring ranges of the
 *               same kind are merged into their bounding range (conservative).
 *   args        args_size <= ACS_ARGS_MAX bytes, the task's argument struct.
 *   seq_out     receives the kernel's submission index (may be NULL).
 * Blocks while the input FIFO is full unless the window is non-blocking.
 * Errors: ACS_EINVAL for an unknown kernel id, args_size too large, a range
 * that wraps past 2^64 (other than the all-memory range), NULL lists with
 * non-zero counts; ACS_EAGAIN when full and non-blocking; ACS_EDEVICE. */
int acs_submit(acs_window *w, int32_t kernel_id,
               const acs_seg *read_segs, int32_t n_read,
               const acs_seg *write_segs, int32_t n_write,
               const void *args, size_t args_size, uint64_t *seq_out);

/* Waits until every submitted kernel has completed: the FIFO and the window
 * are empty, every kernel retired (Section III-C, retirement frees a slot;
 * the program's synchronisation point of Section IV-B).  Returns the first
 * sticky asynchronous error (ACS_EKERNEL, ACS_EDEVICE) if there was one. */
int acs_sync(acs_window *w);

/* As acs_sync (Section III-C, IV-B) but gives up after timeout_ns
 * nanoseconds (ACS_ETIMEDOUT); the window stays usable. */
int acs_sync_timeout(acs_window *w, uint64_t timeout_ns);

/* Window groups, for many independent task graphs in one launch.  With
 * acs_config.n_groups = G > 1 the window is G independent windows of W slots
 * each (the device path needs G * pow2(W) <= 64; G <= 8); acs_submit is
 * acs_submit_group(w, 0, ...).  Kernels of one group are scheduled exactly
 * as in a single window, in their submission order.  Kernels of different
 * groups are never checked against each other: the caller guarantees that
 * no kernel reads or writes bytes that a kernel of another group writes
 * while both can be in flight (graphs on disjoint memory, as separate
 * streams would be).  The in-order and plain paths run all groups through
 * one stream or one host window, which is valid under the same guarantee.
 * Sequence numbers are shared by all groups.  ACS_EINVAL for a group outside
 * [0, G). */
int acs_submit_group(acs_window *w, int32_t group, int32_t kernel_id,
                     const acs_seg *read_segs, int32_t n_read,
                     const acs_seg *write_segs, int32_t n_write,
                     const void *args, size_t args_size, uint64_t *seq_out);

/* Waits until every kernel submitted to `group` has completed (the other
 * groups keep running).  Same return values as acs_sync_timeout (0 = no limit). */
int acs_sync_group(acs_window *w, int32_t group, uint64_t timeout_ns);

/* One non-blocking pass of the host side, for callers that interleave other
 * work with the window (a serving loop): the plain path retires kernels
 * whose completion events fired, admits from the FIFO and launches ready
 * kernels (one turn of the scheduler loop, Algorithm 2); the device and
 * in-order paths have nothing to advance on the host.  Returns the sticky
 * asynchronous error if there is one (ACS_EKERNEL, ACS_EDEVICE), else 0. */
int acs_poll(acs_window *w);

/* Graph capture for a steady state where the same task graph repeats
 * (static networks, repeated requests).  Between acs_graph_begin and
 * acs_graph_end, acs_submit / acs_submit_group record kernels instead of
 * running them (arguments and ranges are checked as usual; sequence numbers
 * advance).  acs_graph_end builds a HIP graph with one kernel node per
 * recorded kernel and an edge from every earlier kernel it conflicts with
 * (the same read/write test as the window, over all pairs, reduced to the
 * edges not implied by others), instantiates it and returns it in *out.
 * The graph borrows the buffers its kernels name: keep them alive until it
 * is destroyed.  Replays see the buffers' contents at launch time.
 * acs_graph_begin: ACS_ESTATE if already recording or the window was stopped.
 * acs_graph_end: ACS_ESTATE if not recording; ACS_EINVAL if nothing was
 * recorded; ACS_EDEVICE if a HIP graph call fails. */
typedef struct acs_graph acs_graph;
int acs_graph_begin(acs_window *w);
int acs_graph_end(acs_window *w, acs_graph **out);
/* Launches one replay on the graph's own stream (asynchronous). */
int acs_graph_launch(acs_graph *g);
/* Waits for every replay launched so far. */
int acs_graph_sync(acs_graph *g);
/* Kernels and dependency edges of the graph. */
int acs_graph_info(const acs_graph *g, int64_t *n_kernels, int64_t *n_edges);
int acs_graph_destroy(acs_graph *g);

/* Copies up to cap entries of the scheduled list into out (oldest first). */
int acs_scheduled_list(acs_window *w, acs_entry *out, int32_t cap, int32_t *n_out);

/* Copies the trace (requires acs_config.trace; call after acs_sync). */
int acs_trace_read(acs_window *w, acs_trace_rec *out, int64_t cap, int64_t *n_out);

int acs_stats_get(acs_window *w, acs_stats *out);

/* Waits for outstanding work and releases the path's execution resources
 * (the device path's persistent kernel exits).  Statistics and the trace stay
 * readable; further submits fail with ACS_ESTATE.  Returns the acs_sync status. */
int acs_window_stop(acs_window *w);

/* Waits for outstanding work (as acs_sync, Section III-C), stops the
 * persistent kernel if any, frees everything the library owns (a window
 * configured without allocation releases its device's static state and
 * leaves the caller's memory and stream alone).  NULL is accepted.
 * Returns the final acs_sync status. */
int acs_window_destroy(acs_window *w);

/* Manual path only: moves up to cap ready kernels (oldest first) to the
 * executing state and returns their seqs. */
int acs_manual_take_ready(acs_window *w, uint64_t *seqs, int32_t cap, int32_t *n_out);
/* Manual path only: reports completion of an executing kernel; status != 0
 * marks it failed, which poisons every kernel that depends on it. */
int acs_manual_complete(acs_window *w, uint64_t seq, int32_t status);

/* What the device path would use on a device (no kernel is launched). */
typedef struct {
    int32_t compute_units;          /* multiprocessor count */
    int32_t wall_clock_khz;         /* constant clock of the device timestamps */
    int32_t persistent_wg_per_cu;   /* resident persistent-kernel workgroups per compute unit */
    int32_t runtime_version;        /* HIP runtime actually loaded in this process */
    int32_t lds_bytes_per_wg;       /* LDS of one persistent-kernel workgroup */
    int32_t reserved[3];
} acs_device_info;

int acs_device_query(int32_t device, acs_device_info *out);

/* Error code of the last failing call on this thread, and its text. */
int acs_last_error(void);
const char *acs_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* ACS_H */
