// fpd_runtime.hip -- host side of the C ABI declared in include/fpdlbm.h.
//
// One fpd_sim owns (or adopts) two population buffers, a device-resident bead state, the
// force-density window of the fiber, a HIP stream and the captured graphs that replay
// chunks of steps.  Every step of the method runs in the kernels of fpd_kernels.hip; this
// file validates, allocates, launches and copies.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stddef.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fpd_internal.hpp"

using namespace fpd;

namespace {

// A roctx range over one call of the C ABI (rocprofv3 --marker-trace shows it beside the
// kernels it launched; without a tool attached the calls return at once).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(FPD_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                            \
    } while (0)

size_t storage_elem(int st) {
    switch (st) {
        case FPD_F64: return 8;
        case FPD_F32: return 4;
        case FPD_F16DEV:
        case FPD_BF16DEV: return 2;
    }
    return 0;
}

int padded_stride(int nx) { return (nx + 63) / 64 * 64; }

int chains_of(const fpd_params* p) { return p->n_chains > 1 ? p->n_chains : 1; }

// Occupancy cells: the smallest power-of-two side >= 32 nodes whose grid fits the bitmap.
void occupancy_cells(int nx, int ny, int& shift, int& cx, int& cy) {
    shift = 5;
    for (;;) {
        cx = (nx + (1 << shift) - 1) >> shift;
        cy = (ny + (1 << shift) - 1) >> shift;
        if ((long long)cx * cy <= 32LL * kOccWords) return;
        ++shift;
    }
}

// Reserved force window (columns, rows): around one fiber, 1.5 times its contour plus the
// support on both sides; several fibers may spread over the whole lattice.
void window_size(const fpd_params* p, double rc, int& w, int& h) {
    if (chains_of(p) > 1) {
        w = p->nx;
        h = p->ny;
        return;
    }
    const double span = 1.5 * (p->n_beads - 1) * p->l0 + 2.0 * rc + 4.0;
    w = (int)ceil(span) < p->nx ? (int)ceil(span) : p->nx;
    h = (int)ceil(span) < p->ny ? (int)ceil(span) : p->ny;
}

// Launch shapes measured best on MI355X at 8192 x 2048 (default block order, no XCD remap):
// 128 x 1 for float64, 256 x 1 for float32, 256 x 1 with two rows per thread for the
// two-byte formats (whose lanes update two nodes each: 512-node tiles).  Below about a
// million nodes the kernel is latency-bound and more, smaller tiles pay: at 1024 x 256,
// 64 x 1 with one row per thread took 15.8 against 17.0 us per step (float32) and 19.9
// against 25.4 (float16 deviations); float64 keeps 128 x 1 (29.8 against 30.3 with 64 x 1).
// nodes = 0: the large-lattice shapes (batches, whose members differ in size).
constexpr long long kSmallLattice = 1LL << 20;

fpd_launch default_launch(int storage, int graph_chunk, long long nodes = 0) {
    const bool small = nodes > 0 && nodes <= kSmallLattice;
    if (storage == FPD_F64) return fpd_launch{128, 1, 1, 2, graph_chunk};
    if (small) return fpd_launch{64, 1, 1, 2, graph_chunk};
    if (nodes_per_lane(storage) > 1) return fpd_launch{256, 1, 2, 2, graph_chunk};
    return fpd_launch{256, 1, 1, 2, graph_chunk};
}

double default_cutoff(int storage) { return storage == FPD_F64 ? 20.0 : 9.0; }

}  // namespace

struct fpd_sim {
    fpd_params p;
    Lattice L;
    size_t elem = 0, buf_bytes = 0;
    void* buf[2] = {nullptr, nullptr};
    bool own_bufs = true;
    int cur = 0;                 // buffer holding the post-collision state of the last step
    hipStream_t stream = nullptr;
    bool own_stream = false;
    BeadState* bs = nullptr;
    void* rect_f = nullptr;
    double* row_phi = nullptr;   // fixed profile phi_s(y) [ny], device (fpd_set_static_phi)
    RecordBuf* rec = nullptr;    // fiber-ends recorder (fpd_record_start)
    int64_t rec_start = 0;       // step count when the recording started
    int rect_wmax = 0, rect_hmax = 0;
    double rc = 0.0;
    bool fiber = false;
    int64_t steps = 0;
    fpd_launch launch{};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_chunk = 0;
    // split steps: the fluid kernels on a side stream, the fiber and bead kernels on
    // `stream`, ordered by the two events (created with the first split step)
    hipStream_t side = nullptr;
    hipEvent_t ev_fluid = nullptr, ev_fiber = nullptr;
    bool part_valid = false;     // BeadState::part[cur] was written by the step before
    // kernel timing
    std::vector<hipEvent_t> events;
    double ms_lat = 0.0, ms_bead = 0.0;
    int64_t n_lat = 0, n_bead = 0;
};

namespace {

StepArgs make_args(const fpd_sim* s, int src_idx) {
    StepArgs a{};
    a.parity = src_idx;
    a.src = s->buf[src_idx];
    a.dst = s->buf[1 - src_idx];
    a.L = s->L;
    a.u6 = s->p.u_wall / 6.0;
    a.gx = s->p.g_body[0];
    a.gy = s->p.g_body[1];
    a.row_phi = s->row_phi;
    a.rec = s->rec;
    const double tau_f = 3.0 * s->p.nu_f + 0.5;
    a.s_nu_f = 1.0 / tau_f;
    a.s_q_f = s->p.s_q_fixed > 0.0 ? s->p.s_q_fixed
                                   : 8.0 * (2.0 - a.s_nu_f) / (8.0 - a.s_nu_f);
    a.s_e = s->p.s_e;
    a.s_eps = s->p.s_eps;
    Fiber& f = a.fib;
    f.bs = s->bs;
    f.n = s->fiber ? s->p.n_beads : 0;
    f.chain_len = s->p.n_beads > 0 ? s->p.n_beads / chains_of(&s->p) : 1;
    occupancy_cells(s->p.nx, s->p.ny, f.occ_shift, f.occ_nx, f.occ_ny);
    f.a = s->p.radius;
    f.xi = s->p.xi;
    f.inv_xi = 1.0 / s->p.xi;
    f.rc = s->rc;
    f.rc2 = s->rc * s->rc;
    f.nu_f = s->p.nu_f;
    f.nu_s = s->p.eta_ratio * s->p.nu_f;
    f.s_q_fixed = s->p.s_q_fixed;
    f.clamp = (s->p.flags & FPD_FLAG_CLAMP_PHI) ? 1 : 0;
    f.rect_f = s->rect_f;
    f.rect_wmax = s->rect_wmax;
    f.rect_hmax = s->rect_hmax;
    f.l0 = s->p.l0;
    f.ks_l02 = s->p.k_s / (s->p.l0 * s->p.l0);
    f.kb = s->p.k_b;
    f.fext[0] = s->p.f_ext[0];
    f.fext[1] = s->p.f_ext[1];
    const fpd_launch& c = s->launch;
    a.rows_per_block = c.block_y * c.rows_per_thread;
    const int tw = c.block_x * nodes_per_lane(s->p.storage);
    a.tiles_x = (s->L.nx + tw - 1) / tw;
    const int tiles_y = (s->L.ny + a.rows_per_block - 1) / a.rows_per_block;
    a.n_tiles = a.tiles_x * tiles_y;
    a.xcd_remap = c.xcd_remap == 1 ? 1 : 0;
    // the fiber kernel's grid holds any partition: a window is at most rect_wmax x
    // rect_hmax nodes, the partition kPartMargin more on each side, and a run of columns
    // meets at most two tiles more than its width in tiles (one may be the narrow last)
    const int m2 = 2 * kPartMargin;
    a.part_gw = std::min(a.tiles_x, (s->rect_wmax + m2 + tw - 1) / tw + 2);
    a.part_gh = std::min(tiles_y, (s->rect_hmax + m2 + a.rows_per_block - 1) / a.rows_per_block + 2);
    return a;
}

int validate(const fpd_params* p) {
    if (!p) return fail(FPD_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1) return fail(FPD_EINVAL, "nx, ny must be >= 1");
    // the row pitch (nine padded direction rows) is a 32-bit element count; offsets of rows
    // are 64-bit, so a buffer may hold more than 2^31 values; the per-row kernels take one
    // grid row per lattice row (at most 65535)
    if (9LL * padded_stride(p->nx) > 0x7fffffffLL)
        return fail(FPD_EINVAL, "nx must stay below 2^31 / 9 (row pitch)");
    if (p->ny > 65535) return fail(FPD_EINVAL, "ny must be at most 65535");
    if (!(p->nu_f > 0.0) || !(3.0 * p->nu_f + 0.5 > 0.5))
        return fail(FPD_EINVAL, "tau_f = 3 nu_f + 1/2 must exceed 1/2 (nu_f = %g)", p->nu_f);
    if (!(fabs(p->u_wall) < 0.1)) return fail(FPD_EINVAL, "|u_wall| must be < 0.1");
    if (!(p->s_e > 0.0 && p->s_e < 2.0) || !(p->s_eps > 0.0 && p->s_eps < 2.0))
        return fail(FPD_EINVAL, "s_e and s_eps must lie in (0, 2)");
    if (p->s_q_fixed > 0.0 && !(p->s_q_fixed < 2.0))
        return fail(FPD_EINVAL, "s_q_fixed must lie in (0, 2)");
    if (storage_elem(p->storage) == 0) return fail(FPD_EINVAL, "unknown storage %d", p->storage);
    if (p->init_flow != FPD_INIT_REST && p->init_flow != FPD_INIT_LINEAR_COUETTE)
        return fail(FPD_EINVAL, "unknown init_flow %d", p->init_flow);
    if (p->n_beads < 0 || p->n_beads > FPD_MAX_BEADS)
        return fail(FPD_EINVAL, "n_beads must be in [0, %d]", FPD_MAX_BEADS);
    if (p->n_chains < 0 || (p->n_beads > 0 && p->n_beads % chains_of(p) != 0))
        return fail(FPD_EINVAL, "n_beads (%d) must be a multiple of n_chains (%d)", p->n_beads,
                    p->n_chains);
    if (p->boundary != FPD_WALLS && p->boundary != FPD_PERIODIC)
        return fail(FPD_EINVAL, "unknown boundary %d", p->boundary);
    if (p->boundary == FPD_PERIODIC && (p->u_wall != 0.0 || p->init_flow != FPD_INIT_REST))
        return fail(FPD_EINVAL, "a periodic box has no walls: u_wall = 0 and FPD_INIT_REST");
    if (!isfinite(p->f_ext[0]) || !isfinite(p->f_ext[1]) || !isfinite(p->g_body[0]) ||
        !isfinite(p->g_body[1]))
        return fail(FPD_EINVAL, "f_ext and g_body must be finite");
    if (!(p->ev_k >= 0.0) || !isfinite(p->ev_k) || !isfinite(p->ev_range))
        return fail(FPD_EINVAL, "ev_k must be finite and >= 0, ev_range finite");
    if (p->n_beads > 0) {
        if (!(p->radius > 0.0) || !(p->xi > 0.0) || !(p->l0 > 0.0))
            return fail(FPD_EINVAL, "radius, xi and l0 must be > 0");
        if (!(p->eta_ratio >= 1.0)) return fail(FPD_EINVAL, "eta_ratio must be >= 1");
        if (!(p->k_s >= 0.0) || !(p->k_b >= 0.0)) return fail(FPD_EINVAL, "k_s, k_b must be >= 0");
    }
    return FPD_OK;
}

int sync_check(fpd_sim* s) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    return FPD_OK;
}

void drop_graphs(fpd_sim* s) {
    for (auto& g : s->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    s->graph_chunk = 0;
}

// The excluded volume between fibers is switched on (then a small kernel sums it before
// every lattice step).
bool has_ev(const fpd_sim* s) {
    return s->fiber && chains_of(&s->p) > 1 && s->p.ev_k > 0.0;
}

// Whether fpd_step splits the lattice step (fluid_kernel / fiber_kernel): with a fiber,
// no fixed profile, not FPD_FLAG_NO_SPLIT, and a fiber kernel grid of at most a quarter
// of the tiles (larger ones leave little to overlap).
// On MI355X at 8192 x 2048 with a 40-bead fiber (graph replay, the fluid kernel's
// occupancy held down as fluid_waves_per_cu states) split steps took about 4 % less than
// whole steps in float64 and float16 deviations and 1 % less in float32: the bead kernel
// runs beside the fluid kernel, less the wait between the two streams (about 5 us against
// 1 us between kernels of one stream).
bool use_split(const fpd_sim* s) {
    if (!s->fiber || s->p.n_beads <= 0 || s->row_phi) return false;
    if (s->p.flags & FPD_FLAG_NO_SPLIT) return false;
    const StepArgs a = make_args(s, s->cur);
    return 4LL * a.part_gw * a.part_gh <= (long long)a.n_tiles;
}

// The side stream and the two events, on the device of the simulation's stream (made
// current for the creation if another one is).
int ensure_split(fpd_sim* s) {
    if (s->side && s->ev_fluid && s->ev_fiber) return FPD_OK;
    hipDevice_t dev = 0;
    int cur = 0;
    HIP_TRY(hipStreamGetDevice(s->stream, &dev));
    HIP_TRY(hipGetDevice(&cur));
    if (dev != cur) HIP_TRY(hipSetDevice(dev));
    hipError_t e = hipSuccess;
    if (!s->side) e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
    if (e == hipSuccess && !s->ev_fluid)
        e = hipEventCreateWithFlags(&s->ev_fluid, hipEventDisableTiming);
    if (e == hipSuccess && !s->ev_fiber)
        e = hipEventCreateWithFlags(&s->ev_fiber, hipEventDisableTiming);
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess)
        return fail(FPD_EDEVICE, "split-step stream or events: %s", hipGetErrorString(e));
    return FPD_OK;
}

// One split step from buffer `from`.  The fluid kernel of step n reads the buffer the
// fluid and fiber kernels of step n - 1 wrote and overwrites the one every kernel of step
// n - 2 read, so it waits for the fiber kernel of step n - 1 (ev_fiber; the fluid kernel
// of n - 1 is before it on the side stream; the bead kernel of n - 2 is before that fiber
// kernel).  The fiber kernel of step n waits for the fluid kernel of step n - 1
// (ev_fluid, taken before it is recorded again) and, on `stream`, for the bead kernel of
// step n - 1, whose positions it needs; the bead kernel of step n reads only tiles of the
// partition, which the fiber kernel wrote.  first: the start of a run (split_steps), whose
// stream is already after every earlier kernel.
int enqueue_split_step(fpd_sim* s, int from, bool first) {
    const StepArgs a = make_args(s, from);
    const dim3 block(s->launch.block_x, s->launch.block_y);
    const int rpt = s->launch.rows_per_thread;
    HIP_TRY(hipStreamWaitEvent(s->side, s->ev_fiber, 0));
    HIP_TRY(launch_step_part(s->p.storage, a, block, rpt, kPartFluid, s->side));
    if (!first) HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_fluid, 0));
    HIP_TRY(hipEventRecord(s->ev_fluid, s->side));
    HIP_TRY(launch_record(a, s->stream));
    if (has_ev(s)) HIP_TRY(launch_ev(a, s->stream));
    HIP_TRY(launch_step_part(s->p.storage, a, block, rpt, kPartFiber, s->stream));
    HIP_TRY(hipEventRecord(s->ev_fiber, s->stream));
    HIP_TRY(launch_bead(s->p.storage, a, 1, 1 - from, s->stream));
    return FPD_OK;
}

// n split steps from buffer `from`, then `stream` waits for the side stream's last kernel,
// so work enqueued on `stream` afterwards follows all of them (also inside a capture, where
// this joins the side stream back).
int split_steps(fpd_sim* s, int from, int64_t n) {
    HIP_TRY(hipEventRecord(s->ev_fiber, s->stream));
    int b = from;
    for (int64_t i = 0; i < n; ++i) {
        int rc = enqueue_split_step(s, b, i == 0);
        if (rc) return rc;
        b = 1 - b;
    }
    HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_fluid, 0));
    return FPD_OK;
}

// One step from buffer `from` (launches only).
int enqueue_step(fpd_sim* s, int from) {
    const StepArgs a = make_args(s, from);
    const dim3 block(s->launch.block_x, s->launch.block_y);
    HIP_TRY(launch_record(a, s->stream));
    if (has_ev(s)) HIP_TRY(launch_ev(a, s->stream));
    HIP_TRY(launch_step(s->p.storage, a, block, s->launch.rows_per_thread, s->stream));
    if (a.fib.n > 0) HIP_TRY(launch_bead(s->p.storage, a, 1, 1 - from, s->stream));
    return FPD_OK;
}

int build_graph(fpd_sim* s, int from, int chunk, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    const bool split = use_split(s);
    if (split) {
        int rs = ensure_split(s);
        if (rs) return rs;
    }
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    int rc = FPD_OK;
    if (split) {
        rc = split_steps(s, from, chunk);
    } else {
        int b = from;
        for (int i = 0; i < chunk && rc == FPD_OK; ++i) {
            rc = enqueue_step(s, b);
            b = 1 - b;
        }
    }
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (rc != FPD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(FPD_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    // move the graph to the device now, so its first replay costs what the others do
    e = hipGraphUpload(*out, s->stream);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "graph upload: %s", hipGetErrorString(e));
    return FPD_OK;
}

// Steps launched one by one, the lattice and bead kernels each stamped with the start and
// end of their own dispatch (durations summed into ms_lat and ms_bead).  Split steps (the
// order of enqueue_split_step) stamp the fluid and the fiber kernel; their lattice pass
// runs from the earlier start to the later end of the two.
int step_timed(fpd_sim* s, int64_t n) {
    const bool fib = s->fiber && s->p.n_beads > 0;
    const bool split = use_split(s);
    if (split) {
        int rc = ensure_split(s);
        if (rc) return rc;
        if (!s->part_valid && n > 0) {  // the first split step's partition (untimed)
            rc = enqueue_step(s, s->cur);
            if (rc) return rc;
            s->cur = 1 - s->cur;
            s->part_valid = true;
            --n;
        }
    }
    const size_t per = split ? 6 : fib ? 4 : 2;
    const dim3 block(s->launch.block_x, s->launch.block_y);
    const int rpt = s->launch.rows_per_thread;
    for (int64_t done = 0; done < n;) {
        const int64_t batch = n - done < 512 ? n - done : 512;
        const size_t need = (size_t)batch * per;
        while (s->events.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            s->events.push_back(e);
        }
        if (split) HIP_TRY(hipEventRecord(s->ev_fiber, s->stream));
        for (int64_t i = 0; i < batch; ++i) {
            const StepArgs a = make_args(s, s->cur);
            hipEvent_t* ev = &s->events[(size_t)i * per];
            if (split) {
                HIP_TRY(hipStreamWaitEvent(s->side, s->ev_fiber, 0));
                HIP_TRY(launch_step_part(s->p.storage, a, block, rpt, kPartFluid, s->side,
                                         ev[0], ev[1]));
                if (i > 0) HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_fluid, 0));
                HIP_TRY(hipEventRecord(s->ev_fluid, s->side));
            }
            HIP_TRY(launch_record(a, s->stream));
            if (has_ev(s)) HIP_TRY(launch_ev(a, s->stream));
            if (split) {
                HIP_TRY(launch_step_part(s->p.storage, a, block, rpt, kPartFiber, s->stream,
                                         ev[2], ev[3]));
                HIP_TRY(hipEventRecord(s->ev_fiber, s->stream));
                HIP_TRY(launch_bead(s->p.storage, a, 1, 1 - s->cur, s->stream, ev[4], ev[5]));
            } else {
                HIP_TRY(launch_step(s->p.storage, a, block, rpt, s->stream, ev[0], ev[1]));
                if (fib)
                    HIP_TRY(launch_bead(s->p.storage, a, 1, 1 - s->cur, s->stream, ev[2],
                                        ev[3]));
            }
            s->cur = 1 - s->cur;
        }
        if (split) HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_fluid, 0));
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (int64_t i = 0; i < batch; ++i) {
            hipEvent_t* ev = &s->events[(size_t)i * per];
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
            if (split) {  // times relative to the fluid kernel's start, either sign
                float fib0 = 0.f, fib1 = 0.f;
                HIP_TRY(hipEventElapsedTime(&fib0, ev[0], ev[2]));
                HIP_TRY(hipEventElapsedTime(&fib1, ev[0], ev[3]));
                ms = std::max(ms, fib1) - std::min(0.f, fib0);
            }
            s->ms_lat += ms;
            s->n_lat += 1;
            if (fib) {
                const hipEvent_t* b = split ? ev + 4 : ev + 2;
                HIP_TRY(hipEventElapsedTime(&ms, b[0], b[1]));
                s->ms_bead += ms;
                s->n_bead += 1;
            }
        }
        done += batch;
    }
    s->part_valid = true;
    return FPD_OK;
}

int fiber_init_device(fpd_sim* s) {
    const StepArgs a = make_args(s, s->cur);
    HIP_TRY(launch_bead(s->p.storage, a, 0, s->cur, s->stream));
    return FPD_OK;
}

int upload_populations(fpd_sim* s, const double* host_f) {
    const size_t n = (size_t)9 * s->p.nx * s->p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    hipError_t e = hipSuccess;
    if (host_f)
        e = hipMemcpyAsync(d, host_f, n * sizeof(double), hipMemcpyHostToDevice, s->stream);
    else
        e = launch_init_eq(s->L, s->p.u_wall, s->p.init_flow, d, s->stream);
    if (e == hipSuccess)
        e = launch_unstream(s->p.storage, s->L, s->p.u_wall, d, s->buf[s->cur], s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "population upload: %s", hipGetErrorString(e));
    return FPD_OK;
}

// Parameters a checkpoint must share with the simulation it is loaded into: everything
// that defines the problem (init_flow only shapes the state a checkpoint replaces, and
// the graph and timing flags can change at any time).
bool params_equal(const fpd_params& a, const fpd_params& b) {
    return a.nx == b.nx && a.ny == b.ny && a.u_wall == b.u_wall && a.nu_f == b.nu_f &&
           a.eta_ratio == b.eta_ratio && a.xi == b.xi && a.n_beads == b.n_beads &&
           a.radius == b.radius && a.l0 == b.l0 && a.k_s == b.k_s && a.k_b == b.k_b &&
           a.s_e == b.s_e && a.s_eps == b.s_eps && a.s_q_fixed == b.s_q_fixed &&
           a.cutoff == b.cutoff && a.storage == b.storage && a.boundary == b.boundary &&
           chains_of(&a) == chains_of(&b) &&
           (a.flags & FPD_FLAG_CLAMP_PHI) == (b.flags & FPD_FLAG_CLAMP_PHI) &&
           a.f_ext[0] == b.f_ext[0] && a.f_ext[1] == b.f_ext[1] &&
           a.g_body[0] == b.g_body[0] && a.g_body[1] == b.g_body[1] && a.ev_k == b.ev_k &&
           a.ev_range == b.ev_range;
}

int create_impl(const fpd_params* p, void* stream, void* fa, void* fb, size_t bytes_each,
                fpd_sim** out) {
    if (!out) return fail(FPD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    fpd_sim* s = new fpd_sim();
    memset(&s->p, 0, sizeof s->p);
    s->p = *p;
    s->L.nx = p->nx;
    s->L.ny = p->ny;
    // the nine direction rows of a lattice row lie side by side: value (k, y, x) sits at
    // y * stride + k * plane + x with plane = padded nx and stride = 9 * plane
    s->L.plane = padded_stride(p->nx);
    s->L.stride = 9 * padded_stride(p->nx);
    s->L.periodic = p->boundary == FPD_PERIODIC ? 1 : 0;
    s->elem = storage_elem(p->storage);
    s->buf_bytes = (size_t)p->ny * (size_t)s->L.stride * s->elem;
    s->rc = p->radius + (p->cutoff > 0.0 ? p->cutoff : default_cutoff(p->storage)) * p->xi;
    s->launch = default_launch(p->storage, 64, (long long)p->nx * p->ny);
    auto bail = [&](int code) {
        fpd_destroy(s);
        return code;
    };
    if (stream) {
        s->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(FPD_EDEVICE, "hipStreamCreate failed"));
        s->own_stream = true;
    }
    if (fa && fb) {
        if (bytes_each < s->buf_bytes)
            return bail(fail(FPD_EINVAL, "buffers of %zu bytes, %zu needed", bytes_each,
                             s->buf_bytes));
        s->buf[0] = fa;
        s->buf[1] = fb;
        s->own_bufs = false;
    } else {
        for (int i = 0; i < 2; ++i)
            if (hipMalloc(&s->buf[i], s->buf_bytes) != hipSuccess) {
                (void)hipGetLastError();
                return bail(fail(FPD_ENOMEM, "hipMalloc of %zu bytes failed", s->buf_bytes));
            }
    }
    // padding columns are never read; clear them once so checkpoints are deterministic
    for (int i = 0; i < 2; ++i)
        if (hipMemsetAsync(s->buf[i], 0, s->buf_bytes, s->stream) != hipSuccess)
            return bail(fail(FPD_EDEVICE, "hipMemset failed"));
    if (hipMalloc((void**)&s->bs, sizeof(BeadState)) != hipSuccess)
        return bail(fail(FPD_ENOMEM, "bead state allocation failed"));
    if (hipMemsetAsync(s->bs, 0, sizeof(BeadState), s->stream) != hipSuccess)
        return bail(fail(FPD_EDEVICE, "hipMemset failed"));
    if (p->n_beads > 0) {
        // window large enough for the chain stretched by 50% in any orientation
        window_size(p, s->rc, s->rect_wmax, s->rect_hmax);
        const size_t tb = p->storage == FPD_F64 ? 8 : 4;
        if (hipMalloc(&s->rect_f, (size_t)s->rect_wmax * s->rect_hmax * 2 * tb) != hipSuccess)
            return bail(fail(FPD_ENOMEM, "fiber window allocation failed"));
        if (hipMemsetAsync(s->rect_f, 0, (size_t)s->rect_wmax * s->rect_hmax * 2 * tb,
                           s->stream) != hipSuccess)
            return bail(fail(FPD_EDEVICE, "hipMemset failed"));
    }
    rc = upload_populations(s, nullptr);
    if (rc) return bail(rc);
    *out = s;
    return FPD_OK;
}

}  // namespace

extern "C" {

const char* fpd_last_error(void) { return g_err.c_str(); }

void fpd_params_default(fpd_params* p) {
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->nx = 64;
    p->ny = 32;
    p->u_wall = 0.0;
    p->nu_f = 1.0 / 6.0;
    p->eta_ratio = 50.0;
    p->xi = 1.0;
    p->n_beads = 0;
    p->radius = 2.0;
    p->l0 = 4.0;
    p->k_s = 0.0;
    p->k_b = 0.0;
    p->s_e = 1.64;
    p->s_eps = 1.54;
    p->s_q_fixed = 0.0;
    p->cutoff = 0.0;
    p->storage = FPD_F32;
    p->init_flow = FPD_INIT_LINEAR_COUETTE;
    p->flags = 0u;
}

int fpd_params_from_physical(double re_ps, double confinement, double kappa, int32_t n_beads,
                             double radius, double eta_ratio, double xi, double u_wall,
                             int32_t nx_over_ny, fpd_params* out) {
    if (!out) return fail(FPD_EINVAL, "out is NULL");
    if (!(re_ps > 0.0) || !(confinement > 0.0 && confinement <= 1.0) || !(kappa >= 0.0) ||
        n_beads < 1 || !(radius > 0.0) || nx_over_ny < 1 || !(u_wall > 0.0))
        return fail(FPD_EINVAL, "physical parameters out of range");
    fpd_params_default(out);
    const double l0 = 2.0 * radius;                        // touching beads, l0 = d
    const double lc = n_beads * l0;                        // contour length
    const int ny = (int)lround(lc / confinement);          // C = l_c / H
    const double gamma = 2.0 * u_wall / ny;                // shear rate of the channel
    const double nu = gamma * lc * lc / (4.0 * re_ps);     // Re_ps = gamma l_c^2 / (4 nu)
    out->nx = nx_over_ny * ny;
    out->ny = ny;
    out->u_wall = u_wall;
    out->nu_f = nu;
    out->eta_ratio = eta_ratio;
    out->xi = xi;
    out->n_beads = n_beads;
    out->radius = radius;
    out->l0 = l0;
    out->k_b = kappa * nu * gamma * lc * lc / 2.0;          // K = 2 k_b / (eta_f gamma l_c^2)
    out->k_s = 0.1 * M_PI * radius * radius * l0 * l0;
    return validate(out);
}

size_t fpd_population_bytes(const fpd_params* p) {
    if (!p || p->nx < 1 || p->ny < 1 || storage_elem(p->storage) == 0) return 0;
    return (size_t)9 * (size_t)p->ny * padded_stride(p->nx) * storage_elem(p->storage);
}

int fpd_create(const fpd_params* p, void* hip_stream, fpd_sim** out) {
    TraceRange range("fpd_create");
    return create_impl(p, hip_stream, nullptr, nullptr, 0, out);
}

int fpd_create_with_buffers(const fpd_params* p, void* hip_stream, void* f_a, void* f_b,
                            size_t bytes_each, fpd_sim** out) {
    TraceRange range("fpd_create_with_buffers");
    if (!f_a || !f_b) return fail(FPD_EINVAL, "buffers must not be NULL");
    if (((uintptr_t)f_a | (uintptr_t)f_b) & 15)
        return fail(FPD_EINVAL, "buffers must be 16-byte aligned");
    return create_impl(p, hip_stream, f_a, f_b, bytes_each, out);
}

void fpd_destroy(fpd_sim* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->side) (void)hipStreamSynchronize(s->side);
    drop_graphs(s);
    for (auto e : s->events) (void)hipEventDestroy(e);
    if (s->ev_fluid) (void)hipEventDestroy(s->ev_fluid);
    if (s->ev_fiber) (void)hipEventDestroy(s->ev_fiber);
    if (s->side) (void)hipStreamDestroy(s->side);
    if (s->own_bufs)
        for (auto& b : s->buf)
            if (b) (void)hipFree(b);
    if (s->bs) (void)hipFree(s->bs);
    if (s->rect_f) (void)hipFree(s->rect_f);
    if (s->row_phi) (void)hipFree(s->row_phi);
    if (s->rec) (void)hipFree(s->rec);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int fpd_init_fiber(fpd_sim* s, const double* R) {
    if (!s || !R) return fail(FPD_EINVAL, "NULL argument");
    const int N = s->p.n_beads;
    if (N <= 0) return fail(FPD_ESTATE, "the simulation was created without beads");
    for (int i = 0; i < N; ++i) {
        const double x = R[2 * i], y = R[2 * i + 1];
        if (!isfinite(x) || !isfinite(y)) return fail(FPD_EINVAL, "bead %d is not finite", i);
        if (s->p.boundary == FPD_WALLS &&
            (y - s->p.radius - s->p.xi < 0.0 || y + s->p.radius + s->p.xi > s->p.ny))
            return fail(FPD_EINVAL, "bead %d lies within a + xi of a wall", i);
    }
    const int Lc = N / chains_of(&s->p);
    for (int i = 0; i + 1 < N; ++i) {
        if ((i + 1) % Lc == 0) continue;  // last bead of a fiber: no bond to the next one
        const double dx = R[2 * i + 2] - R[2 * i], dy = R[2 * i + 3] - R[2 * i + 1];
        const double span = sqrt(dx * dx + dy * dy);
        if (!(span > 0.0)) return fail(FPD_EINVAL, "beads %d and %d coincide", i, i + 1);
    }
    // extent check against the reserved window (the device re-checks every step)
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int i = 0; i < N; ++i) {
        xmin = fmin(xmin, R[2 * i]);
        xmax = fmax(xmax, R[2 * i]);
        ymin = fmin(ymin, R[2 * i + 1]);
        ymax = fmax(ymax, R[2 * i + 1]);
    }
    if ((xmax - xmin) + 2.0 * s->rc + 3.0 > s->rect_wmax && s->rect_wmax < s->p.nx)
        return fail(FPD_EINVAL, "fiber extent exceeds 1.5 (N-1) l0");
    if ((ymax - ymin) + 2.0 * s->rc + 3.0 > s->rect_hmax && s->rect_hmax < s->p.ny)
        return fail(FPD_EINVAL, "fiber extent exceeds 1.5 (N-1) l0");
    int rc0 = sync_check(s);
    if (rc0) return rc0;
    BeadState h;
    memset(&h, 0, sizeof h);
    HIP_TRY(hipMemcpy(&h, s->bs, sizeof h, hipMemcpyDeviceToHost));
    for (int i = 0; i < N; ++i) {
        h.R[i][0] = R[2 * i];
        h.R[i][1] = R[2 * i + 1];
        h.V[i][0] = h.V[i][1] = 0.0;
    }
    memset(h.occ, 0, sizeof h.occ);  // empty occupancy; the bead kernel fills slot `cur`
    h.ev_k = chains_of(&s->p) > 1 ? s->p.ev_k : 0.0;  // one fiber: nothing to exclude
    h.ev_d = s->p.ev_range > 0.0 ? s->p.ev_range : 2.0 * s->p.radius;
    for (int k = 0; k < 2; ++k) {  // empty windows; the bead kernel fills slot `cur`
        h.win[k][0] = 0x7fffffff;
        h.win[k][1] = -0x7fffffff;
        h.win[k][2] = 0x7fffffff;
        h.win[k][3] = -0x7fffffff;
    }
    HIP_TRY(hipMemcpyAsync(s->bs, &h, sizeof h, hipMemcpyHostToDevice, s->stream));
    drop_graphs(s);
    s->part_valid = false;
    s->fiber = true;  // make_args hands the beads to the kernels only with a fiber
    // the stream is synchronised on every path below: the copy reads h from this frame
    const int rc = fiber_init_device(s);
    const int rs = sync_check(s);
    if (rc || rs) {
        s->fiber = false;
        return rc ? rc : rs;
    }
    return FPD_OK;
}

int fpd_init_fiber_line(fpd_sim* s, double cx, double cy, double theta) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    const int N = s->p.n_beads;
    if (N <= 0) return fail(FPD_ESTATE, "the simulation was created without beads");
    std::vector<double> R(2 * (size_t)N);
    for (int i = 1; i <= N; ++i) {
        const double t = (i - (N + 1) / 2.0) * s->p.l0;
        R[2 * (i - 1)] = cx + t * cos(theta);
        R[2 * (i - 1) + 1] = cy + t * sin(theta);
    }
    return fpd_init_fiber(s, R.data());
}

}  // extern "C"

namespace {

// Whether n steps from buffer `from` replay graphs, and the graph they replay captured
// (nothing runs).
int ensure_graph(fpd_sim* s, int from, int64_t n, bool* replay) {
    const int chunk = s->launch.graph_chunk;
    *replay = !(s->p.flags & (FPD_FLAG_NO_GRAPH | FPD_FLAG_TIME_KERNELS)) && chunk >= 2 &&
              n >= chunk;
    if (!*replay) return FPD_OK;
    if (s->graph_chunk != chunk) {
        drop_graphs(s);
        s->graph_chunk = chunk;
    }
    if (!s->graph[from]) return build_graph(s, from, chunk, &s->graph[from]);
    return FPD_OK;
}

}  // namespace

extern "C" {

int fpd_capture(fpd_sim* s, int64_t n) {
    TraceRange range("fpd_capture");
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    if (n < 0) return fail(FPD_EINVAL, "n_steps must be >= 0");
    if (s->p.n_beads > 0 && !s->fiber)
        return fail(FPD_ESTATE, "fpd_init_fiber must come before fpd_capture");
    bool replay = false;
    if (use_split(s) && !s->part_valid && n > 0)  // fpd_step runs one whole step first
        return ensure_graph(s, 1 - s->cur, n - 1, &replay);
    return ensure_graph(s, s->cur, n, &replay);
}

int fpd_step(fpd_sim* s, int64_t n) {
    TraceRange range("fpd_step");
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    if (n < 0) return fail(FPD_EINVAL, "n_steps must be >= 0");
    if (n == 0) return FPD_OK;
    if (s->p.n_beads > 0 && !s->fiber)
        return fail(FPD_ESTATE, "fpd_init_fiber must come before fpd_step");
    const uint32_t fl = s->p.flags;
    if (fl & FPD_FLAG_TIME_KERNELS) {
        int rc = step_timed(s, n);
        if (rc) return rc;
        s->steps += n;
        return FPD_OK;
    }
    int64_t left = n;
    const bool split = use_split(s);
    if (split) {
        int rc = ensure_split(s);
        if (rc) return rc;
        if (!s->part_valid) {  // the first split step's partition comes from a whole step
            rc = enqueue_step(s, s->cur);
            if (rc) return rc;
            s->cur = 1 - s->cur;
            s->part_valid = true;
            --left;
        }
    }
    const int chunk = s->launch.graph_chunk;
    bool replay = false;
    int rg = ensure_graph(s, s->cur, left, &replay);
    if (rg) return rg;
    if (replay) {
        while (left >= chunk) {
            HIP_TRY(hipGraphLaunch(s->graph[s->cur], s->stream));
            left -= chunk;  // chunk is even: the state returns to the same buffer
        }
    }
    if (left > 0 && split) {
        int rc = split_steps(s, s->cur, left);
        if (rc) return rc;
        if (left & 1) s->cur = 1 - s->cur;
        left = 0;
    }
    for (; left > 0; --left) {
        int rc = enqueue_step(s, s->cur);
        if (rc) return rc;
        s->cur = 1 - s->cur;
    }
    s->steps += n;
    s->part_valid = true;
    return FPD_OK;
}

int fpd_sync(fpd_sim* s) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    int rc = sync_check(s);
    if (rc) return rc;
    if (s->fiber) {
        unsigned h = 0;
        HIP_TRY(hipMemcpy(&h, &s->bs->health, sizeof h, hipMemcpyDeviceToHost));
        if (h) return fail(FPD_EUNSTABLE, "health flags 0x%x", h);
    }
    return FPD_OK;
}

int fpd_health(fpd_sim* s, uint32_t* flags, double* max_strain) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    int rc = sync_check(s);
    if (rc) return rc;
    unsigned h = 0;
    unsigned long long bits = 0;
    HIP_TRY(hipMemcpy(&h, &s->bs->health, sizeof h, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&bits, &s->bs->max_strain_bits, sizeof bits, hipMemcpyDeviceToHost));
    double ms;
    memcpy(&ms, &bits, sizeof ms);
    if (flags) *flags = h;
    if (max_strain) *max_strain = ms;
    return FPD_OK;
}

int fpd_clear_health(fpd_sim* s) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    int rc = sync_check(s);
    if (rc) return rc;
    const unsigned zero = 0;
    const unsigned long long zbits = 0;
    HIP_TRY(hipMemcpy(&s->bs->health, &zero, sizeof zero, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(&s->bs->max_strain_bits, &zbits, sizeof zbits, hipMemcpyHostToDevice));
    return FPD_OK;
}

int fpd_step_count(fpd_sim* s, int64_t* steps) {
    if (!s || !steps) return fail(FPD_EINVAL, "NULL argument");
    *steps = s->steps;
    return FPD_OK;
}

int fpd_read_fields(fpd_sim* s, double* rho, double* ux, double* uy, double* eta) {
    TraceRange range("fpd_read_fields");
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    const size_t S = (size_t)s->p.nx * s->p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, 4 * S * sizeof(double)));
    const StepArgs a = make_args(s, s->cur);
    hipError_t e = launch_forces(a, s->stream);  // C = F / A of the current bead state
    if (e == hipSuccess)
        e = launch_fields(s->p.storage, a, d, d + S, d + 2 * S, d + 3 * S, s->stream);
    double* outs[4] = {rho, ux, uy, eta};
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
        if (outs[i])
            e = hipMemcpyAsync(outs[i], d + i * S, S * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "read_fields: %s", hipGetErrorString(e));
    return FPD_OK;
}

int fpd_set_static_phi(fpd_sim* s, const double* phi) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    const int ny = s->p.ny;
    if (phi)
        for (int j = 0; j < ny; ++j)
            if (!isfinite(phi[j]) || phi[j] < 0.0)
                return fail(FPD_EINVAL, "phi_s[%d] must be finite and >= 0", j);
    int rc = sync_check(s);
    if (rc) return rc;
    if (!phi) {
        if (s->row_phi) (void)hipFree(s->row_phi);
        s->row_phi = nullptr;
    } else {
        if (!s->row_phi && hipMalloc((void**)&s->row_phi, sizeof(double) * ny) != hipSuccess) {
            (void)hipGetLastError();
            s->row_phi = nullptr;
            return fail(FPD_ENOMEM, "static profile allocation failed");
        }
        HIP_TRY(hipMemcpy(s->row_phi, phi, sizeof(double) * ny, hipMemcpyHostToDevice));
    }
    drop_graphs(s);  // the captured arguments name the profile
    return FPD_OK;
}

int fpd_record_start(fpd_sim* s, int32_t every, int64_t capacity) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    if (s->p.n_beads <= 0) return fail(FPD_ESTATE, "the simulation has no fiber");
    if (every < 1 || capacity < 1 || capacity > (1LL << 28))
        return fail(FPD_EINVAL, "every >= 1 and 1 <= capacity <= 2^28 required");
    int rc = sync_check(s);
    if (rc) return rc;
    if (s->rec) (void)hipFree(s->rec);
    s->rec = nullptr;
    const int fibers = chains_of(&s->p);
    const size_t bytes = offsetof(RecordBuf, data) +
                         sizeof(double) * (size_t)capacity * (size_t)(1 + 4 * fibers);
    if (hipMalloc((void**)&s->rec, bytes) != hipSuccess) {
        (void)hipGetLastError();
        s->rec = nullptr;
        return fail(FPD_ENOMEM, "recorder allocation failed");
    }
    RecordBuf h;
    memset(&h, 0, sizeof h);
    h.every = every;
    h.cap = (int)capacity;
    h.fibers = fibers;
    HIP_TRY(hipMemcpy(s->rec, &h, offsetof(RecordBuf, data), hipMemcpyHostToDevice));
    s->rec_start = s->steps;
    drop_graphs(s);  // the captured arguments name the recorder
    return FPD_OK;
}

int fpd_record_stop(fpd_sim* s) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    int rc = sync_check(s);
    if (rc) return rc;
    if (s->rec) (void)hipFree(s->rec);
    s->rec = nullptr;
    drop_graphs(s);
    return FPD_OK;
}

int fpd_record_read(fpd_sim* s, double* out, int64_t cap, int64_t* n) {
    if (!s || !n) return fail(FPD_EINVAL, "NULL argument");
    if (!s->rec) return fail(FPD_ESTATE, "no recording");
    int rc = sync_check(s);
    if (rc) return rc;
    RecordBuf h;
    HIP_TRY(hipMemcpy(&h, s->rec, offsetof(RecordBuf, data), hipMemcpyDeviceToHost));
    const int64_t taken = (int64_t)((h.count + h.every - 1) / (unsigned long long)h.every);
    const int64_t have = taken < h.cap ? taken : h.cap;
    *n = have;
    if (!out || have == 0) return FPD_OK;
    if (cap < have)
        return fail(FPD_EINVAL, "output holds %lld records, %lld needed", (long long)cap,
                    (long long)have);
    const int width = 1 + 4 * h.fibers;
    std::vector<double> ring((size_t)h.cap * width);
    HIP_TRY(hipMemcpy(ring.data(), (char*)s->rec + offsetof(RecordBuf, data),
                      sizeof(double) * ring.size(), hipMemcpyDeviceToHost));
    const int64_t first = taken - have;  // oldest record still held
    for (int64_t k = 0; k < have; ++k) {
        const double* src = ring.data() + (size_t)((first + k) % h.cap) * width;
        double* dst = out + (size_t)k * width;
        dst[0] = src[0] + (double)s->rec_start;  // absolute step of the state R^n
        for (int j = 1; j < width; ++j) dst[j] = src[j];
    }
    return FPD_OK;
}

int fpd_particle_stats(fpd_sim* s, int32_t bead, double* out) {
    if (!s || !out) return fail(FPD_EINVAL, "NULL argument");
    if (!s->fiber || bead < 0 || bead >= s->p.n_beads)
        return fail(FPD_EINVAL, "no bead %d in this simulation", bead);
    int rc0 = sync_check(s);
    if (rc0) return rc0;
    double R[2];
    HIP_TRY(hipMemcpy(R, &s->bs->R[bead][0], sizeof R, hipMemcpyDeviceToHost));
    if (!isfinite(R[0]) || !isfinite(R[1]) || fabs(R[0]) > 1e9 || fabs(R[1]) > 1e9)
        return fail(FPD_EUNSTABLE, "bead %d is not at a finite position", bead);
    const int nx = s->p.nx, ny = s->p.ny;
    auto wrap = [](long long v, int n) { long long r = v % n; return (int)(r < 0 ? r + n : r); };
    // the support box grown by one node (where grad phi can be non-zero) plus a one-node
    // border for the stencil
    const long long xlo = (long long)floor(R[0] - 0.5 - s->rc) - 2;
    const long long xhi = (long long)ceil(R[0] - 0.5 + s->rc) + 2;
    const long long ylo = (long long)floor(R[1] - 0.5 - s->rc) - 2;
    const long long yhi = (long long)ceil(R[1] - 0.5 + s->rc) + 2;
    NodeBox B;
    if (xhi - xlo + 1 >= nx) {
        B.cx0 = 0;
        B.cw = nx;
        B.wrap_x = true;
    } else {
        B.cx0 = wrap(xlo, nx);
        B.cw = (int)(xhi - xlo + 1);
        B.wrap_x = false;
    }
    if (s->p.boundary == FPD_PERIODIC) {
        if (yhi - ylo + 1 >= ny) {
            B.cy0 = 0;
            B.ch = ny;
            B.wrap_y = true;
        } else {
            B.cy0 = wrap(ylo, ny);
            B.ch = (int)(yhi - ylo + 1);
            B.wrap_y = false;
        }
    } else {
        if (ylo < 0 || yhi > ny - 1)
            return fail(FPD_EINVAL, "bead %d is too close to a wall for the diagnostics", bead);
        B.cy0 = (int)ylo;
        B.ch = (int)(yhi - ylo + 1);
        B.wrap_y = false;
    }
    double* d = nullptr;
    const size_t n = (size_t)B.cw * (size_t)B.ch;
    HIP_TRY(hipMalloc(&d, (4 * n + 8) * sizeof(double)));
    const StepArgs a = make_args(s, s->cur);
    hipError_t e = launch_forces(a, s->stream);  // C = F / A of the current bead state
    if (e == hipSuccess)
        e = launch_particle_stats(s->p.storage, a, bead, B, d, d + 4 * n, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d + 4 * n, 8 * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "particle_stats: %s", hipGetErrorString(e));
    return FPD_OK;
}

int fpd_read_populations(fpd_sim* s, double* f) {
    TraceRange range("fpd_read_populations");
    if (!s || !f) return fail(FPD_EINVAL, "NULL argument");
    const size_t n = (size_t)9 * s->p.nx * s->p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    hipError_t e = launch_stream_out(s->p.storage, s->L, s->p.u_wall, s->buf[s->cur], d, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "read_populations: %s", hipGetErrorString(e));
    return FPD_OK;
}

int fpd_write_populations(fpd_sim* s, const double* f) {
    if (!s || !f) return fail(FPD_EINVAL, "NULL argument");
    int rc = sync_check(s);
    if (rc) return rc;
    return upload_populations(s, f);
}

// R, V and F are read with one copy
constexpr size_t kBeadPairs = sizeof(double) * 2 * kMaxBeads;
static_assert(offsetof(BeadState, V) == offsetof(BeadState, R) + kBeadPairs &&
                  offsetof(BeadState, F) == offsetof(BeadState, V) + kBeadPairs,
              "R, V, F must be adjacent in BeadState");

int fpd_read_beads(fpd_sim* s, double* R, double* V, double* F) {
    TraceRange range("fpd_read_beads");
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    const int N = s->p.n_beads;
    if (N == 0) return FPD_OK;
    HIP_TRY(launch_forces(make_args(s, s->cur), s->stream));  // F^n of the current positions
    int rc = sync_check(s);
    if (rc) return rc;
    std::vector<double> h(2 * (size_t)kMaxBeads * 3);
    HIP_TRY(hipMemcpy(h.data(), s->bs->R, sizeof(double) * 2 * kMaxBeads * 3,
                      hipMemcpyDeviceToHost));
    for (int i = 0; i < N; ++i)
        for (int c = 0; c < 2; ++c) {
            if (R) R[2 * i + c] = h[2 * i + c];
            if (V) V[2 * i + c] = h[2 * kMaxBeads + 2 * i + c];
            if (F) F[2 * i + c] = h[4 * kMaxBeads + 2 * i + c];
        }
    return FPD_OK;
}

}  // extern "C"

namespace {

// `cur` with the fields of `c` that are > 0, checked against the shapes the lattice
// kernels are built for.
int merge_launch(const fpd_launch& cur, const fpd_launch* c, fpd_launch& n) {
    n = cur;
    if (c->block_x > 0) n.block_x = c->block_x;
    if (c->block_y > 0) n.block_y = c->block_y;
    if (c->rows_per_thread > 0) n.rows_per_thread = c->rows_per_thread;
    if (c->xcd_remap > 0) n.xcd_remap = c->xcd_remap;
    if (c->graph_chunk > 0) n.graph_chunk = c->graph_chunk;
    if (n.block_x != 64 && n.block_x != 128 && n.block_x != 256)
        return fail(FPD_EINVAL, "block_x must be 64, 128 or 256");
    if (n.block_y != 1 && n.block_y != 2 && n.block_y != 4)
        return fail(FPD_EINVAL, "block_y must be 1, 2 or 4");
    if (n.block_x * n.block_y > 256) return fail(FPD_EINVAL, "at most 256 threads per block");
    if (n.rows_per_thread != 1 && n.rows_per_thread != 2 && n.rows_per_thread != 4)
        return fail(FPD_EINVAL, "rows_per_thread must be 1, 2 or 4");
    if (n.xcd_remap != 1 && n.xcd_remap != 2) return fail(FPD_EINVAL, "xcd_remap must be 1 or 2");
    if (n.graph_chunk < 2 || (n.graph_chunk & 1))
        return fail(FPD_EINVAL, "graph_chunk must be even and >= 2");
    return FPD_OK;
}

}  // namespace

extern "C" {

int fpd_set_launch(fpd_sim* s, const fpd_launch* c) {
    if (!s || !c) return fail(FPD_EINVAL, "NULL argument");
    fpd_launch n;
    int rc = merge_launch(s->launch, c, n);
    if (rc) return rc;
    rc = sync_check(s);
    if (rc) return rc;
    s->launch = n;
    drop_graphs(s);
    return FPD_OK;
}

int fpd_set_flags(fpd_sim* s, uint32_t flags) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    int rc = sync_check(s);
    if (rc) return rc;
    const uint32_t keep = s->p.flags & FPD_FLAG_CLAMP_PHI;
    s->p.flags =
        keep | (flags & (FPD_FLAG_NO_GRAPH | FPD_FLAG_TIME_KERNELS | FPD_FLAG_NO_SPLIT));
    drop_graphs(s);
    return FPD_OK;
}

int fpd_split_active(fpd_sim* s, int32_t* on) {
    if (!s || !on) return fail(FPD_EINVAL, "NULL argument");
    *on = use_split(s) ? 1 : 0;
    return FPD_OK;
}

int fpd_get_launch(fpd_sim* s, fpd_launch* c) {
    if (!s || !c) return fail(FPD_EINVAL, "NULL argument");
    *c = s->launch;
    return FPD_OK;
}

int fpd_kernel_times(fpd_sim* s, double* ms_lattice, int64_t* n_lattice, double* ms_bead,
                     int64_t* n_bead) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    if (ms_lattice) *ms_lattice = s->ms_lat;
    if (n_lattice) *n_lattice = s->n_lat;
    if (ms_bead) *ms_bead = s->ms_bead;
    if (n_bead) *n_bead = s->n_bead;
    return FPD_OK;
}

int fpd_reset_kernel_times(fpd_sim* s) {
    if (!s) return fail(FPD_EINVAL, "NULL simulation");
    s->ms_lat = s->ms_bead = 0.0;
    s->n_lat = s->n_bead = 0;
    return FPD_OK;
}

int fpd_copy_probe(void* hip_stream, size_t bytes, int32_t iters, double* gbps) {
    if (bytes == 0 || (bytes & 15) || iters < 1 || !gbps)
        return fail(FPD_EINVAL, "bytes must be a positive multiple of 16, iters >= 1");
    hipStream_t st = (hipStream_t)hip_stream;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return fail(FPD_ENOMEM, "copy probe allocation");
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipFree(a);
        return fail(FPD_ENOMEM, "copy probe allocation");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, bytes, st);
    if (e == hipSuccess) e = launch_copy(a, b, bytes, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < iters && e == hipSuccess; ++i) e = launch_copy(a, b, bytes, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "copy probe: %s", hipGetErrorString(e));
    *gbps = 2.0 * (double)bytes * iters / (ms * 1e-3) / 1e9;
    return FPD_OK;
}

// ---------------------------------------------------------------- checkpoint -------

static const char kMagic[8] = {'F', 'P', 'D', 'L', 'B', 'M', '0', '7'};

int fpd_save(fpd_sim* s, const char* path) {
    TraceRange range("fpd_save");
    if (!s || !path) return fail(FPD_EINVAL, "NULL argument");
    int rc = sync_check(s);
    if (rc) return rc;
    std::vector<char> pops(s->buf_bytes);
    BeadState h;
    HIP_TRY(hipMemcpy(pops.data(), s->buf[s->cur], s->buf_bytes, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&h, s->bs, sizeof h, hipMemcpyDeviceToHost));
    FILE* fp = fopen(path, "wb");
    if (!fp) return fail(FPD_EINVAL, "cannot open %s for writing", path);
    const uint8_t fib = s->fiber ? 1 : 0;
    const uint8_t par = (uint8_t)s->cur;  // the bead state's window slot follows the parity
    bool ok = fwrite(kMagic, 1, 8, fp) == 8 && fwrite(&s->p, sizeof s->p, 1, fp) == 1 &&
              fwrite(&s->steps, sizeof s->steps, 1, fp) == 1 && fwrite(&fib, 1, 1, fp) == 1 &&
              fwrite(&par, 1, 1, fp) == 1 &&
              fwrite(&s->buf_bytes, sizeof s->buf_bytes, 1, fp) == 1 &&
              fwrite(pops.data(), 1, pops.size(), fp) == pops.size() &&
              fwrite(&h, sizeof h, 1, fp) == 1;
    ok = (fclose(fp) == 0) && ok;
    if (!ok) return fail(FPD_EDEVICE, "write to %s failed", path);
    return FPD_OK;
}

int fpd_load(fpd_sim* s, const char* path) {
    TraceRange range("fpd_load");
    if (!s || !path) return fail(FPD_EINVAL, "NULL argument");
    int rc = sync_check(s);
    if (rc) return rc;
    FILE* fp = fopen(path, "rb");
    if (!fp) return fail(FPD_EINVAL, "cannot open %s", path);
    char magic[8];
    fpd_params p;
    int64_t steps = 0;
    uint8_t fib = 0, par = 0;
    size_t bytes = 0;
    bool ok = fread(magic, 1, 8, fp) == 8 && memcmp(magic, kMagic, 8) == 0 &&
              fread(&p, sizeof p, 1, fp) == 1 && fread(&steps, sizeof steps, 1, fp) == 1 &&
              fread(&fib, 1, 1, fp) == 1 && fread(&par, 1, 1, fp) == 1 && par <= 1 &&
              fread(&bytes, sizeof bytes, 1, fp) == 1;
    if (!ok || bytes != s->buf_bytes || !params_equal(p, s->p)) {
        fclose(fp);
        return fail(FPD_EINVAL, "%s does not match this simulation", path);
    }
    std::vector<char> pops(bytes);
    BeadState h;
    ok = fread(pops.data(), 1, bytes, fp) == bytes && fread(&h, sizeof h, 1, fp) == 1;
    fclose(fp);
    if (!ok) return fail(FPD_EINVAL, "%s is truncated", path);
    drop_graphs(s);
    s->part_valid = false;
    s->cur = par;
    HIP_TRY(hipMemcpy(s->buf[s->cur], pops.data(), bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->bs, &h, sizeof h, hipMemcpyHostToDevice));
    s->steps = steps;
    s->fiber = fib != 0;
    return FPD_OK;
}

}  // extern "C"

// ==================================================================== batches ====

namespace {

struct BatchEntry {
    fpd_sim* sim = nullptr;
    int64_t id = 0;
    int64_t remaining = 0;
    int status = FPD_SIM_ACTIVE;
    bool reported = false;
    size_t bytes = 0;
};

}  // namespace

struct fpd_batch {
    size_t budget = 0, used = 0;
    int max_slots = 0, storage = FPD_F32;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    fpd_launch launch{};
    std::vector<BatchEntry> entries;
    int64_t next_id = 1;
    // device work tables and their pinned host mirrors
    StepArgs* d_args = nullptr;
    int* d_counts = nullptr;
    BeadState** d_states = nullptr;
    unsigned* d_health = nullptr;
    StepArgs* h_args = nullptr;
    int* h_tile_off = nullptr;
    int* h_bead_off = nullptr;
    int* h_counts = nullptr;
    BeadState** h_states = nullptr;
    unsigned* h_health = nullptr;
    ItemRef* d_tile_items = nullptr;   // item tables (device, pinned host)
    ItemRef* d_bead_items = nullptr;
    ItemRef* h_tile_items = nullptr;
    ItemRef* h_bead_items = nullptr;
    int cap_tiles = 0, cap_beads = 0;
    std::vector<int> table;  // entry index of table row r
    bool dirty = true;
    bool pending = false;        // steps enqueued by fpd_batch_launch, not yet waited for
    int64_t pending_steps = 0;
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 0;
    int graph_counts[3] = {0, 0, 0};  // counts the graph's grids were sized for
    bool any_periodic = false;        // some active simulation has no walls
    bool graph_periodic = false;      // the kernel variant the graph was captured with
};

namespace {

void batch_drop_graph(fpd_batch* b) {
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_chunk = 0;
}

BatchEntry* find_entry(fpd_batch* b, int64_t id) {
    for (auto& e : b->entries)
        if (e.id == id) return &e;
    return nullptr;
}

size_t footprint_of(const fpd_params* p) {
    const size_t pop = fpd_population_bytes(p);
    size_t rect = 0;
    if (p->n_beads > 0) {
        const double rc = p->radius + (p->cutoff > 0.0 ? p->cutoff : default_cutoff(p->storage)) * p->xi;
        int w = 0, h = 0;
        window_size(p, rc, w, h);
        rect = (size_t)w * (size_t)h * 2 * (p->storage == FPD_F64 ? 8 : 4);
    }
    return 2 * pop + rect + sizeof(BeadState);
}

// Rebuild the work tables for the active simulations (call with the stream idle).
int batch_rebuild(fpd_batch* b) {
    b->table.clear();
    int tiles = 0, beads = 0, r = 0;
    b->h_tile_off[0] = 0;
    b->h_bead_off[0] = 0;
    for (size_t i = 0; i < b->entries.size(); ++i) {
        BatchEntry& e = b->entries[i];
        if (e.status != FPD_SIM_ACTIVE || e.remaining <= 0) continue;
        fpd_sim* s = e.sim;
        b->h_args[2 * r] = make_args(s, s->cur);
        b->h_args[2 * r + 1] = make_args(s, 1 - s->cur);
        tiles += b->h_args[2 * r].n_tiles;
        beads += b->h_args[2 * r].fib.n;
        b->h_tile_off[r + 1] = tiles;
        b->h_bead_off[r + 1] = beads;
        b->h_states[r] = s->bs;
        b->table.push_back((int)i);
        ++r;
    }
    b->h_counts[0] = r;
    b->h_counts[1] = tiles;
    b->h_counts[2] = beads;
    b->any_periodic = false;
    for (int q = 0; q < r; ++q)
        if (b->h_args[2 * q].L.periodic) b->any_periodic = true;
    if (b->graph && (b->graph_counts[0] != r || b->graph_counts[1] != tiles ||
                     b->graph_counts[2] != beads || b->graph_periodic != b->any_periodic))
        batch_drop_graph(b);  // its grids or kernel variant no longer match the tables
    // item tables (grown geometrically; a new pointer drops the graph)
    auto grow = [&](int need, int& cap, ItemRef*& d, ItemRef*& h) -> int {
        if (need <= cap) return FPD_OK;
        int ncap = cap > 0 ? cap : 1024;
        while (ncap < need) ncap *= 2;
        if (d) (void)hipFree(d);
        if (h) (void)hipHostFree(h);
        d = nullptr;
        h = nullptr;
        cap = 0;
        if (hipMalloc((void**)&d, sizeof(ItemRef) * ncap) != hipSuccess ||
            hipHostMalloc((void**)&h, sizeof(ItemRef) * ncap, 0) != hipSuccess)
            return fail(FPD_ENOMEM, "batch item table allocation failed");
        cap = ncap;
        batch_drop_graph(b);
        return FPD_OK;
    };
    int rc = grow(tiles, b->cap_tiles, b->d_tile_items, b->h_tile_items);
    if (rc == FPD_OK) rc = grow(beads, b->cap_beads, b->d_bead_items, b->h_bead_items);
    if (rc) return rc;
    for (int q = 0; q < r; ++q) {
        for (int t = b->h_tile_off[q]; t < b->h_tile_off[q + 1]; ++t)
            b->h_tile_items[t] = ItemRef{q, t - b->h_tile_off[q]};
        for (int t = b->h_bead_off[q]; t < b->h_bead_off[q + 1]; ++t)
            b->h_bead_items[t] = ItemRef{q, t - b->h_bead_off[q]};
    }
    if (tiles > 0)
        HIP_TRY(hipMemcpyAsync(b->d_tile_items, b->h_tile_items, sizeof(ItemRef) * tiles,
                               hipMemcpyHostToDevice, b->stream));
    if (beads > 0)
        HIP_TRY(hipMemcpyAsync(b->d_bead_items, b->h_bead_items, sizeof(ItemRef) * beads,
                               hipMemcpyHostToDevice, b->stream));
    if (r > 0) {
        HIP_TRY(hipMemcpyAsync(b->d_args, b->h_args, sizeof(StepArgs) * 2 * r,
                               hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->d_states, b->h_states, sizeof(BeadState*) * r,
                               hipMemcpyHostToDevice, b->stream));
    }
    HIP_TRY(hipMemcpyAsync(b->d_counts, b->h_counts, sizeof(int) * 3, hipMemcpyHostToDevice,
                           b->stream));
    b->dirty = false;
    return FPD_OK;
}

int batch_enqueue(fpd_batch* b, int gpar) {
    BatchArgs a{b->d_args, b->d_tile_items, b->d_bead_items, b->d_counts, gpar};
    const dim3 block(b->launch.block_x, b->launch.block_y);
    HIP_TRY(launch_batch_step(b->storage, a, block, b->launch.rows_per_thread, b->h_counts,
                              b->any_periodic, b->stream));
    return FPD_OK;
}

int batch_build_graph(fpd_batch* b, int chunk) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = FPD_OK;
    for (int i = 0; i < chunk && rc == FPD_OK; ++i) rc = batch_enqueue(b, i & 1);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc != FPD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(FPD_EDEVICE, "batch graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "batch graph instantiate: %s", hipGetErrorString(e));
    e = hipGraphUpload(b->graph, b->stream);
    if (e != hipSuccess) return fail(FPD_EDEVICE, "batch graph upload: %s", hipGetErrorString(e));
    b->graph_chunk = chunk;
    for (int k = 0; k < 3; ++k) b->graph_counts[k] = b->h_counts[k];
    b->graph_periodic = b->any_periodic;
    return FPD_OK;
}

}  // namespace

extern "C" {

size_t fpd_sim_footprint(const fpd_params* p) {
    if (!p || validate(p) != FPD_OK) return 0;
    return footprint_of(p);
}

// FPD_EINVAL while steps enqueued by fpd_batch_launch await fpd_batch_wait.
static int batch_idle(const fpd_batch* b) {
    if (b->pending) return fail(FPD_EINVAL, "a launch is pending: call fpd_batch_wait first");
    return FPD_OK;
}

int fpd_batch_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t storage,
                     void* hip_stream, fpd_batch** out) {
    if (!out) return fail(FPD_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096) return fail(FPD_EINVAL, "max_slots must be in 1..4096");
    if (storage_elem(storage) == 0) return fail(FPD_EINVAL, "unknown storage %d", storage);
    fpd_batch* b = new fpd_batch();
    b->budget = hbm_budget_bytes;
    b->max_slots = max_slots;
    b->storage = storage;
    b->launch = default_launch(storage, 32);
    auto bail = [&](int code) {
        fpd_batch_destroy(b);
        return code;
    };
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(FPD_EDEVICE, "hipStreamCreate failed"));
        b->own_stream = true;
    }
    const size_t n = (size_t)max_slots;
    bool ok = hipMalloc((void**)&b->d_args, sizeof(StepArgs) * 2 * n) == hipSuccess &&
              hipMalloc((void**)&b->d_counts, sizeof(int) * 3) == hipSuccess &&
              hipMalloc((void**)&b->d_states, sizeof(BeadState*) * n) == hipSuccess &&
              hipMalloc((void**)&b->d_health, sizeof(unsigned) * n) == hipSuccess &&
              hipHostMalloc((void**)&b->h_args, sizeof(StepArgs) * 2 * n, 0) == hipSuccess &&
              hipHostMalloc((void**)&b->h_tile_off, sizeof(int) * (n + 1), 0) == hipSuccess &&
              hipHostMalloc((void**)&b->h_bead_off, sizeof(int) * (n + 1), 0) == hipSuccess &&
              hipHostMalloc((void**)&b->h_counts, sizeof(int) * 3, 0) == hipSuccess &&
              hipHostMalloc((void**)&b->h_states, sizeof(BeadState*) * n, 0) == hipSuccess &&
              hipHostMalloc((void**)&b->h_health, sizeof(unsigned) * n, 0) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return bail(fail(FPD_ENOMEM, "batch table allocation failed"));
    }
    int rc = batch_rebuild(b);
    if (rc) return bail(rc);
    *out = b;
    return FPD_OK;
}

void fpd_batch_destroy(fpd_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (auto& e : b->entries) fpd_destroy(e.sim);
    b->entries.clear();
    (void)hipFree(b->d_args);
    (void)hipFree(b->d_counts);
    (void)hipFree(b->d_states);
    (void)hipFree(b->d_health);
    (void)hipFree(b->d_tile_items);
    (void)hipFree(b->d_bead_items);
    (void)hipHostFree(b->h_tile_items);
    (void)hipHostFree(b->h_bead_items);
    (void)hipHostFree(b->h_args);
    (void)hipHostFree(b->h_tile_off);
    (void)hipHostFree(b->h_bead_off);
    (void)hipHostFree(b->h_counts);
    (void)hipHostFree(b->h_states);
    (void)hipHostFree(b->h_health);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int fpd_batch_set_launch(fpd_batch* b, const fpd_launch* c) {
    if (!b || !c) return fail(FPD_EINVAL, "NULL argument");
    if (b->pending) return batch_idle(b);
    fpd_launch n;
    int rc = merge_launch(b->launch, c, n);  // checked before any member changes
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (auto& e : b->entries) {
        rc = fpd_set_launch(e.sim, &n);
        if (rc) return rc;
    }
    b->launch = n;
    batch_drop_graph(b);
    b->dirty = true;
    return FPD_OK;
}

int fpd_batch_add(fpd_batch* b, const fpd_params* p, const double* R, int64_t n_steps,
                  int64_t* sim_id) {
    TraceRange range("fpd_batch_add");
    if (!b || !p || !sim_id) return fail(FPD_EINVAL, "NULL argument");
    if (b->pending) return batch_idle(b);
    if (n_steps < 0) return fail(FPD_EINVAL, "n_steps must be >= 0");
    int rc = validate(p);
    if (rc) return rc;
    if (p->storage != b->storage) return fail(FPD_EINVAL, "storage differs from the batch's");
    if (p->n_beads > 0 && !R) return fail(FPD_EINVAL, "bead positions are required");
    const size_t need = footprint_of(p);
    if ((int)b->entries.size() >= b->max_slots) return fail(FPD_ENOMEM, "no free slot");
    if (b->used + need > b->budget)
        return fail(FPD_ENOMEM, "HBM budget: %zu + %zu > %zu bytes", b->used, need, b->budget);
    HIP_TRY(hipStreamSynchronize(b->stream));
    fpd_sim* s = nullptr;
    rc = create_impl(p, b->stream, nullptr, nullptr, 0, &s);
    if (rc) return rc;
    rc = fpd_set_launch(s, &b->launch);
    if (rc == FPD_OK && p->n_beads > 0) rc = fpd_init_fiber(s, R);
    if (rc) {
        fpd_destroy(s);
        return rc;
    }
    BatchEntry e;
    e.sim = s;
    e.id = b->next_id++;
    e.remaining = n_steps;
    e.status = n_steps == 0 ? FPD_SIM_DONE : FPD_SIM_ACTIVE;
    e.bytes = need;
    b->entries.push_back(e);
    b->used += need;
    b->dirty = true;
    *sim_id = e.id;
    return FPD_OK;
}

int fpd_batch_launch(fpd_batch* b, int64_t max_steps, int64_t* advanced) {
    TraceRange range("fpd_batch_launch");
    if (!b) return fail(FPD_EINVAL, "NULL batch");
    if (advanced) *advanced = 0;
    int rc = batch_idle(b);
    if (rc) return rc;
    if (max_steps <= 0) return FPD_OK;
    int64_t steps = max_steps;
    int active = 0;
    for (auto& e : b->entries)
        if (e.status == FPD_SIM_ACTIVE && e.remaining > 0) {
            ++active;
            if (e.remaining < steps) steps = e.remaining;
        }
    if (active == 0) return FPD_OK;
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->dirty) {
        rc = batch_rebuild(b);
        if (rc) return rc;
    }
    int64_t left = steps;
    const int chunk = b->launch.graph_chunk;
    if (left >= chunk) {
        if (b->graph_chunk != chunk) {
            batch_drop_graph(b);
            rc = batch_build_graph(b, chunk);
            if (rc) return rc;
        }
        while (left >= chunk) {
            HIP_TRY(hipGraphLaunch(b->graph, b->stream));
            left -= chunk;
        }
    }
    for (int i = 0; left > 0; --left, ++i) {
        rc = batch_enqueue(b, i & 1);
        if (rc) return rc;
    }
    // health of every simulation, read back once the steps are done
    const int rows = (int)b->table.size();
    HIP_TRY(health_gather(b->d_states, b->d_health, rows, b->stream));
    if (rows > 0)
        HIP_TRY(hipMemcpyAsync(b->h_health, b->d_health, sizeof(unsigned) * rows,
                               hipMemcpyDeviceToHost, b->stream));
    b->pending = true;
    b->pending_steps = steps;
    if (advanced) *advanced = steps;
    return FPD_OK;
}

int fpd_batch_wait(fpd_batch* b) {
    TraceRange range("fpd_batch_wait");
    if (!b) return fail(FPD_EINVAL, "NULL batch");
    if (!b->pending) return FPD_OK;
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->pending = false;
    const int64_t steps = b->pending_steps;
    b->pending_steps = 0;
    const int rows = (int)b->table.size();
    for (int r = 0; r < rows; ++r) {
        BatchEntry& e = b->entries[b->table[r]];
        e.remaining -= steps;
        e.sim->steps += steps;
        if (steps & 1) e.sim->cur ^= 1;
        if (b->h_health[r]) {
            e.status = FPD_SIM_FAILED;
        } else if (e.remaining == 0) {
            e.status = FPD_SIM_DONE;
        }
        if (e.status != FPD_SIM_ACTIVE) b->dirty = true;
    }
    if (steps & 1) b->dirty = true;
    return FPD_OK;
}

int fpd_batch_run(fpd_batch* b, int64_t max_steps, int64_t* advanced) {
    const int rc = fpd_batch_launch(b, max_steps, advanced);
    if (rc) return rc;
    return fpd_batch_wait(b);
}

int fpd_batch_poll(fpd_batch* b, int64_t* ids, int32_t* status, int32_t cap, int32_t* n) {
    if (!b || !n) return fail(FPD_EINVAL, "NULL argument");
    int k = 0;
    for (auto& e : b->entries) {
        if (k >= cap) break;
        if (e.status != FPD_SIM_ACTIVE && !e.reported) {
            if (ids) ids[k] = e.id;
            if (status) status[k] = e.status;
            e.reported = true;
            ++k;
        }
    }
    *n = k;
    return FPD_OK;
}

int fpd_batch_read_beads(fpd_batch* b, int64_t id, double* R, double* V, double* F) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    return fpd_read_beads(e->sim, R, V, F);
}

int fpd_batch_read_populations(fpd_batch* b, int64_t id, double* f) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    return fpd_read_populations(e->sim, f);
}

int fpd_batch_read_fields(fpd_batch* b, int64_t id, double* rho, double* ux, double* uy,
                          double* eta) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    return fpd_read_fields(e->sim, rho, ux, uy, eta);
}

int fpd_batch_set_static_phi(fpd_batch* b, int64_t id, const double* phi) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int rc = fpd_set_static_phi(e->sim, phi);
    if (rc == FPD_OK) b->dirty = true;  // the argument table names the profile
    return rc;
}

int fpd_batch_record_start(fpd_batch* b, int64_t id, int32_t every, int64_t capacity) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int rc = fpd_record_start(e->sim, every, capacity);
    if (rc == FPD_OK) b->dirty = true;  // the argument table names the recorder
    return rc;
}

int fpd_batch_record_read(fpd_batch* b, int64_t id, double* out, int64_t cap, int64_t* n) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    HIP_TRY(hipStreamSynchronize(b->stream));
    return fpd_record_read(e->sim, out, cap, n);
}

int fpd_batch_particle_stats(fpd_batch* b, int64_t id, int32_t bead, double* out) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    return fpd_particle_stats(e->sim, bead, out);
}

int fpd_batch_sim_info(fpd_batch* b, int64_t id, int64_t* steps, int32_t* status,
                       uint32_t* health) {
    if (b && b->pending) return batch_idle(b);
    BatchEntry* e = b ? find_entry(b, id) : nullptr;
    if (!e) return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
    if (steps) *steps = e->sim->steps;
    if (status) *status = e->status;
    if (health) {
        double ms;
        int rc = fpd_health(e->sim, health, &ms);
        if (rc) return rc;
    }
    return FPD_OK;
}

int fpd_batch_release(fpd_batch* b, int64_t id) {
    TraceRange range("fpd_batch_release");
    if (!b) return fail(FPD_EINVAL, "NULL batch");
    if (b->pending) return batch_idle(b);
    for (size_t i = 0; i < b->entries.size(); ++i)
        if (b->entries[i].id == id) {
            HIP_TRY(hipStreamSynchronize(b->stream));
            fpd_destroy(b->entries[i].sim);
            b->used -= b->entries[i].bytes;
            b->entries.erase(b->entries.begin() + (long)i);
            b->dirty = true;
            return FPD_OK;
        }
    return fail(FPD_EINVAL, "unknown simulation %lld", (long long)id);
}

int fpd_batch_stats(fpd_batch* b, int32_t* active, int32_t* held, size_t* bytes_in_use) {
    if (!b) return fail(FPD_EINVAL, "NULL batch");
    int a = 0;
    for (auto& e : b->entries)
        if (e.status == FPD_SIM_ACTIVE) ++a;
    if (active) *active = a;
    if (held) *held = (int)b->entries.size();
    if (bytes_in_use) *bytes_in_use = b->used;
    return FPD_OK;
}

}  // extern "C"

// ------------------------------------------------------- allocation-free entry ----
//
// fpd_run_static runs one simulation on caller-owned population buffers with the bead
// state and the force-density window in `scratch`, a file-scope device array of fixed
// size: it calls no allocator.  Each device holds its own copy of the array (at its own
// address, looked up once per device with hipGetSymbolAddress) until the process ends, and
// every call on a device shares it.

static __device__ __align__(256) unsigned char scratch[FPD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kScratchBeadBytes = (sizeof(BeadState) + 255) / 256 * 256;
static_assert(FPD_STATIC_SCRATCH_BYTES % 256 == 0 &&
                  kScratchBeadBytes < (size_t)FPD_STATIC_SCRATCH_BYTES,
              "the bead state must fit the static scratch array");

std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Device address of this device's scratch array (the host-side name is only a stand-in).
int scratch_ptr(unsigned char** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FPD_EDEVICE, "device %d beyond the %d the static scratch supports", dev,
                    kMaxDevices);
    std::call_once(g_scratch_once[dev], [dev] {
        g_scratch_err[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
        return fail(FPD_EDEVICE, "hipGetSymbolAddress(scratch): %s",
                    hipGetErrorString(g_scratch_err[dev]));
    *out = (unsigned char*)g_scratch_ptr[dev];
    return FPD_OK;
}

}  // namespace

extern "C" {

size_t fpd_static_scratch_need(const fpd_params* p) {
    if (!p || p->n_beads <= 0) return 0;
    const double rc = p->radius + (p->cutoff > 0.0 ? p->cutoff : default_cutoff(p->storage)) *
                                      p->xi;
    int w = 0, h = 0;
    window_size(p, rc, w, h);
    const size_t tb = p->storage == FPD_F64 ? 8 : 4;
    return kScratchBeadBytes + (size_t)w * (size_t)h * 2 * tb;
}

int fpd_run_static(const fpd_params* p, void* hip_stream, void* f_a, void* f_b,
                   size_t bytes_each, int32_t init_populations, const double* R_in,
                   double* R_out, uint32_t* health, int64_t n_steps) {
    TraceRange range("fpd_run_static");
    int rc = validate(p);
    if (rc) return rc;
    if (n_steps < 0) return fail(FPD_EINVAL, "n_steps must be >= 0");
    if (!f_a || !f_b) return fail(FPD_EINVAL, "buffers must not be NULL");
    if (((uintptr_t)f_a | (uintptr_t)f_b) & 15)
        return fail(FPD_EINVAL, "buffers must be 16-byte aligned");
    const size_t need_buf = fpd_population_bytes(p);
    if (bytes_each < need_buf)
        return fail(FPD_EINVAL, "buffers of %zu bytes, %zu needed", bytes_each, need_buf);
    const int N = p->n_beads;
    if (N > 0 && (!R_in || !R_out)) return fail(FPD_EINVAL, "R_in and R_out are required");
    const size_t need = fpd_static_scratch_need(p);
    if (need > (size_t)FPD_STATIC_SCRATCH_BYTES)
        return fail(FPD_EINVAL,
                    "bead state and force window need %zu bytes of static scratch; the "
                    "maximum is %zu (FPD_STATIC_SCRATCH_BYTES)",
                    need, (size_t)FPD_STATIC_SCRATCH_BYTES);
    unsigned char* base = nullptr;
    rc = scratch_ptr(&base);
    if (rc) return rc;

    // a simulation record on the stack: nothing below allocates
    fpd_sim s;
    s.p = *p;
    s.L.nx = p->nx;
    s.L.ny = p->ny;
    s.L.plane = padded_stride(p->nx);
    s.L.stride = 9 * padded_stride(p->nx);
    s.L.periodic = p->boundary == FPD_PERIODIC ? 1 : 0;
    s.elem = storage_elem(p->storage);
    s.buf_bytes = need_buf;
    s.buf[0] = f_a;
    s.buf[1] = f_b;
    s.own_bufs = false;
    s.cur = 0;
    s.stream = (hipStream_t)hip_stream;
    s.rc = p->radius + (p->cutoff > 0.0 ? p->cutoff : default_cutoff(p->storage)) * p->xi;
    s.launch = default_launch(p->storage, 64, (long long)p->nx * p->ny);
    if (init_populations)
        HIP_TRY(launch_init_state(p->storage, s.L, p->u_wall, p->init_flow, f_a, s.stream));
    if (N > 0) {
        s.bs = (BeadState*)base;
        s.rect_f = base + kScratchBeadBytes;
        window_size(p, s.rc, s.rect_wmax, s.rect_hmax);
        // the state a new simulation starts from: everything zero (the earlier call's
        // contents are not used), then the fiber as fpd_init_fiber sets it
        HIP_TRY(launch_zero(base, need, s.stream));
        const double ev_k = chains_of(p) > 1 ? p->ev_k : 0.0;
        const double ev_d = p->ev_range > 0.0 ? p->ev_range : 2.0 * p->radius;
        HIP_TRY(launch_fiber_setup(s.bs, R_in, N, ev_k, ev_d, s.stream));
        s.fiber = true;
        HIP_TRY(launch_bead(p->storage, make_args(&s, 0), 0, 0, s.stream));
    }
    for (int64_t i = 0; i < n_steps; ++i) {
        rc = enqueue_step(&s, s.cur);
        if (rc) return rc;
        s.cur = 1 - s.cur;
    }
    if (N > 0 || health) HIP_TRY(launch_beads_out(s.bs, N, R_out, health, s.stream));
    return FPD_OK;
}

}  // extern "C"
