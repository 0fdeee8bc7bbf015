// api.hip -- the extern "C" entry points of igg.h: argument checks (all on
// the host, before any HIP call), the implicit global grid state (one rank,
// or several virtual ranks as blocks on this device), the boundary-first
// schedule of the steps, the time loop with its captured graph, and kernel
// timing.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "host.hpp"

namespace igg {

static thread_local std::string t_last_error;

int fail(int code, const std::string &msg)
{
    t_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return fail(IGG_ERR_HIP, buf);
}

Grid &grid()
{
    static Grid g;
    return g;
}

int64_t zmarch_min_points() { return grid().zmarch_min; }

void rank_coords(int r, int c[3])
{
    const Grid &g = grid();
    c[0] = r % g.dims[0];
    c[1] = (r / g.dims[0]) % g.dims[1];
    c[2] = r / (g.dims[0] * g.dims[1]);
}

int rank_neighbor(int r, int d, int side)
{
    const Grid &g = grid();
    int c[3];
    rank_coords(r, c);
    c[d] += side ? 1 : -1;
    if (c[d] < 0 || c[d] >= g.dims[d]) {
        if (!g.periods[d]) return -1;
        c[d] = (c[d] + g.dims[d]) % g.dims[d];
    }
    return c[0] + g.dims[0] * (c[1] + g.dims[1] * c[2]);
}

int elem_bytes(int dtype) { return dtype == IGG_F64 ? 8 : dtype == IGG_F32 ? 4 : 2; }

int64_t field_elems(const igg_field &f) { return f.size[0] * f.size[1] * f.size[2]; }

bool overlaps_mem(const igg_field &a, const igg_field &b)
{
    uintptr_t a0 = (uintptr_t)a.data, a1 = a0 + (uintptr_t)(field_elems(a) * elem_bytes(a.dtype));
    uintptr_t b0 = (uintptr_t)b.data, b1 = b0 + (uintptr_t)(field_elems(b) * elem_bytes(b.dtype));
    return a0 < b1 && b0 < a1;
}

int check_field(const igg_field *f, const char *name, bool grid_sized)
{
    Grid &g = grid();
    if (!f) return fail(IGG_ERR_ARG, std::string(name) + ": null field");
    if (!f->data) return fail(IGG_ERR_ARG, std::string(name) + ": null data pointer");
    if (f->reserved != 0) return fail(IGG_ERR_ARG, std::string(name) + ": reserved must be 0");
    if (f->dtype < IGG_F64 || f->dtype > IGG_F16)
        return fail(IGG_ERR_DTYPE, std::string(name) + ": unknown dtype " + std::to_string(f->dtype));
    for (int d = 0; d < 3; ++d) {
        int64_t s = f->size[d];
        bool ok = grid_sized ? (s == g.n[d]) : (s == g.n[d] || s == g.n[d] + 1);
        if (!ok) {
            char buf[256];
            snprintf(buf, sizeof buf, "%s: size (%lld,%lld,%lld) does not fit the grid (%d,%d,%d)%s",
                     name, (long long)f->size[0], (long long)f->size[1], (long long)f->size[2],
                     g.n[0], g.n[1], g.n[2], grid_sized ? "" : " (n or n+1 per dimension)");
            return fail(IGG_ERR_SIZE, buf);
        }
    }
    return IGG_OK;
}

static int check_finite_pos(double v, const char *name, bool allow_zero)
{
    if (!isfinite(v) || v < 0.0 || (!allow_zero && v == 0.0))
        return fail(IGG_ERR_ARG, std::string(name) + " must be finite and " +
                                     (allow_zero ? "non-negative" : "positive"));
    return IGG_OK;
}

int plan_split(const int n[3], const int w[3], Split &s)
{
    s.nb = 0;
    int kz0 = std::min(w[2], n[2] - 1), kz1 = std::max(n[2] - w[2], kz0);
    int jy0 = std::min(w[1], n[1] - 1), jy1 = std::max(n[1] - w[1], jy0);
    int ix0 = std::min(w[0], n[0] - 1), ix1 = std::max(n[0] - w[0], ix0);
    auto add = [&](int kind, int i0, int i1, int j0, int j1, int k0, int k1) {
        if (i0 < i1 && j0 < j1 && k0 < k1) {
            s.kind[s.nb] = kind;
            s.boundary[s.nb++] = Box{i0, i1, j0, j1, k0, k1};
        }
    };
    const int X = n[0] - 1, Y = n[1] - 1, Z = n[2] - 1;
    add(1, 1, X, 1, Y, 1, kz0);        // z low slab
    add(1, 1, X, 1, Y, kz1, Z);        // z high slab
    add(1, 1, X, 1, jy0, kz0, kz1);    // y low slab
    add(1, 1, X, jy1, Y, kz0, kz1);    // y high slab
    add(0, 1, ix0, jy0, jy1, kz0, kz1);  // x low slab
    add(0, ix1, X, jy0, jy1, kz0, kz1);  // x high slab
    s.inner = Box{ix0, ix1, jy0, jy1, kz0, kz1};
    return IGG_OK;
}

BoxSet make_boxset(const Box *b, int nb)
{
    BoxSet bs{};
    bs.n = nb;
    int64_t t = 0;
    for (int q = 0; q < nb; ++q) {
        int w = b[q].i1 - b[q].i0;
        int lg = 3;
        while ((1 << lg) < w && lg < 6) ++lg;
        bs.b[q] = b[q];
        bs.lpr_log2[q] = lg;
        bs.nseg_x[q] = (w + (1 << lg) - 1) >> lg;
        bs.first[q] = t;
        t += (int64_t)bs.nseg_x[q] * (b[q].j1 - b[q].j0) * (b[q].k1 - b[q].k0) << lg;
    }
    for (int q = nb; q < 7; ++q) bs.first[q] = t;
    return bs;
}

uint32_t sr_key(uint64_t seed, uint64_t counter)
{
    uint32_t h = pcg_hash((uint32_t)(counter >> 32));
    h = pcg_hash((uint32_t)counter ^ h);
    h = pcg_hash((uint32_t)(seed >> 32) ^ h);
    return pcg_hash((uint32_t)seed ^ h);
}

int ensure_device()
{
    Grid &g = grid();
    int dev = -1;
    IGG_HIP(hipGetDevice(&dev));
    if (g.dev_ready) {
        if (dev != g.device)
            return fail(IGG_ERR_ARG, "the grid's GPU resources live on device " + std::to_string(g.device) +
                                         ", current device is " + std::to_string(dev));
        return IGG_OK;
    }
    // default priority: the helper stream is an ordinary second stream
    IGG_HIP(hipStreamCreateWithFlags(&g.side, hipStreamNonBlocking));
    // fork/join events order work between two streams of this device only:
    // no timing and no system-scope fence (a fence writes back the caches
    // at every record, tens of microseconds per step at 512^3)
    IGG_HIP(hipEventCreateWithFlags(&g.ev_fork, hipEventDisableTiming | hipEventDisableSystemFence));
    IGG_HIP(hipEventCreateWithFlags(&g.ev_join, hipEventDisableTiming | hipEventDisableSystemFence));
    // one plane of the largest field (n+1 per dimension) in FP64, rounded to 256 B
    int64_t m0 = (int64_t)(g.n[1] + 1) * (g.n[2] + 1), m1 = (int64_t)(g.n[0] + 1) * (g.n[2] + 1),
            m2 = (int64_t)(g.n[0] + 1) * (g.n[1] + 1);
    int64_t cap = std::max(m0, std::max(m1, m2)) * 8;
    g.halo_cap = (size_t)((cap + 255) / 256 * 256);
    IGG_HIP(hipMalloc((void **)&g.halo_buf, g.halo_cap * 2 * 2 * IGG_MAX_FIELDS * g.nranks));
    IGG_HIP(hipMalloc((void **)&g.red_part, 8192 * sizeof(double)));
    IGG_HIP(hipHostMalloc((void **)&g.red_host, 64 * sizeof(double), hipHostMallocDefault));
    g.device = dev;
    g.dev_ready = true;
    return IGG_OK;
}

static int release_device()
{
    Grid &g = grid();
    if (!g.dev_ready) return IGG_OK;
    int rc = IGG_OK;
    auto chk = [&](hipError_t e, const char *w) {
        if (e != hipSuccess && rc == IGG_OK) rc = hip_fail(e, w);
    };
    chk(hipStreamSynchronize(g.side), "hipStreamSynchronize(side)");
    chk(hipFree(g.halo_buf), "hipFree(halo_buf)");
    chk(hipFree(g.red_part), "hipFree(red_part)");
    chk(hipHostFree(g.red_host), "hipHostFree(red_host)");
    chk(hipEventDestroy(g.ev_fork), "hipEventDestroy");
    chk(hipEventDestroy(g.ev_join), "hipEventDestroy");
    for (hipEvent_t e : g.tev) chk(hipEventDestroy(e), "hipEventDestroy(timing)");
    chk(hipStreamDestroy(g.side), "hipStreamDestroy(side)");
    if (g.run_exec) chk(hipGraphExecDestroy(g.run_exec), "hipGraphExecDestroy");
    if (g.cap) chk(hipStreamDestroy(g.cap), "hipStreamDestroy(cap)");
    g.run_exec = nullptr;
    g.cap = nullptr;
    g.run_key.clear();
    g.tev.clear();
    g.dev_ready = false;
    return rc;
}

// events made when timing is switched on: 1024 timed launches
static const size_t kTimingPool = 2048;

// Bracket a launch on stream s with timing events when timing is enabled;
// kind 0 marks the inner-region kernel, kind 1 the boundary kernels.
static int timing_mark(hipStream_t s, int kind)
{
    Grid &g = grid();
    if (!g.timing) return IGG_OK;
    if (g.tev_used == g.tev.size()) {
        // timing only: no system-scope fence, which would add a cache
        // write-back to the work being timed
        hipEvent_t e;
        IGG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        g.tev.push_back(e);
        g.tev_kind.push_back(0);
    }
    g.tev_kind[g.tev_used] = kind;
    IGG_HIP(hipEventRecord(g.tev[g.tev_used++], s));
    return IGG_OK;
}

static int64_t box_points(const Box &b)
{
    return (int64_t)std::max(0, b.i1 - b.i0) * std::max(0, b.j1 - b.j0) * std::max(0, b.k1 - b.k0);
}

// A fixed-length wait on one wavefront, `iters` rounds of the longest
// s_sleep: put into one stream by the IGG_TEST_DELAY setting, it lets a test
// hold back one side of the boundary-first schedule and check that the
// events between the streams, not the timing, order the work.
__global__ void k_test_delay(int iters)
{
    for (int q = 0; q < iters; ++q) __builtin_amdgcn_s_sleep(127);
}

static int test_delay(int where, hipStream_t s)
{
    Grid &g = grid();
    if (g.delay_where != where || g.delay_iters <= 0) return IGG_OK;
    hipLaunchKernelGGL(k_test_delay, dim3(1), dim3(64), 0, s, g.delay_iters);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

// inner regions of at least this many points run the boundary slabs and the
// halo update on the helper stream by default, smaller ones in one chain on
// the caller stream
static const int64_t kSideMinPoints = (int64_t)1 << 21;

static int check_split(const int *split, const int *ol)
{
    if (!split) return IGG_OK;
    for (int d = 0; d < 3; ++d)
        if (split[d] < ol[d])
            return fail(IGG_ERR_ARG, "split width " + std::to_string(split[d]) + " in dimension " +
                                         std::to_string(d) + " is below the overlap " +
                                         std::to_string(ol[d]));
    return IGG_OK;
}

static int check_spacings(double lam, double dt, double dx, double dy, double dz)
{
    int rc;
    if ((rc = check_finite_pos(lam, "lam", false))) return rc;
    if ((rc = check_finite_pos(dt, "dt", true))) return rc;
    if ((rc = check_finite_pos(dx, "dx", false))) return rc;
    if ((rc = check_finite_pos(dy, "dy", false))) return rc;
    if ((rc = check_finite_pos(dz, "dz", false))) return rc;
    return IGG_OK;
}

// One step with boundary-first split: the slabs the halo update reads, then
// the update of `out`.  Schedule 1 runs both on the helper stream while the
// inner region runs on the caller stream (as hide_communication does with
// its boundary streams); schedule 0 runs the slabs on the caller stream ahead
// of the inner region and only the update beside it; schedule 2 runs slabs,
// update and inner region in that order on the caller stream; schedule 3
// (where the caller provides fused_launch) runs the slabs and the inner
// region in one launch whose first work-groups take the slabs, and then
// whatever halo update is left.  By default a caller with fused_launch (the
// one-rank periodic step, whose slab kernel stores the y and z halo itself)
// takes schedule 3: at 512^3 it is 0.8-2.6% faster than the unsplit step
// while schedules 1 and 2 are slower, the slabs beside the inner launch
// costing more bandwidth than the update they hide.  Otherwise large inner
// regions take schedule 1; small grids are launch-bound, the cross-stream
// fork and join cost more than the update they would hide, and a captured
// graph of a single chain replays fastest, so they take schedule 2.  FP16
// fields take schedule 2 at any size, as do callers whose inner kernel is
// partly latency-bound (the adjoint passes side_ok = false): its slabs
// beside the inner region cost 5.5% at 256^3 and 2% at 512^3.  When the x
// exchange is fused into the stores (or x is not periodic) the update never
// reads the x slabs, so they join the inner launch and the boundary phase is
// the y and z slabs.
// boundary(r, slabs, stream) and inner(r, box, stream) launch rank r's
// kernels, halo(stream) the halo update of the results.
template <typename HaloLaunch, typename BoundaryLaunch, typename InnerLaunch>
static int run_split(const int *split, int dtype, HaloLaunch halo, BoundaryLaunch boundary,
                     InnerLaunch inner_launch, hipStream_t s, bool side_ok = true,
                     int (*fused_launch)(int, const Split &, const Box &, hipStream_t, void *) = nullptr,
                     void *fused_ctx = nullptr)
{
    Grid &g = grid();
    int rc;
    Split sp;
    plan_split(g.n, split, sp);
    Split bnd = sp;
    Box inner = sp.inner;
    if (g.fuse_x) {
        bnd.nb = 0;
        for (int q = 0; q < sp.nb; ++q) {
            if (sp.kind[q] == 0) continue;
            bnd.boundary[bnd.nb] = sp.boundary[q];
            bnd.kind[bnd.nb++] = sp.kind[q];
        }
        inner.i0 = 1;
        inner.i1 = g.n[0] - 1;
    }
    const bool side_pays = side_ok && box_points(inner) >= kSideMinPoints && dtype != IGG_F16;
    int sched = g.schedule >= 0 ? g.schedule : (fused_launch ? 3 : side_pays ? 1 : 2);
    if (sched == 3 && !fused_launch) sched = 2;
    if (sched == 3) {
        // one launch: the slab work-groups first, then the inner tiles; the
        // halo update (if any is left after the fused pack) follows it
        for (int r = 0; r < g.nranks; ++r) {
            if ((rc = timing_mark(s, 0))) return rc;
            if ((rc = fused_launch(r, bnd, inner, s, fused_ctx))) return rc;
            if ((rc = timing_mark(s, 0))) return rc;
            if (g.timing) {
                g.t_launches++;
                g.t_points += box_points(inner);
                for (int q = 0; q < bnd.nb; ++q) g.t_points += box_points(bnd.boundary[q]);
            }
        }
        if ((rc = test_delay(3, s))) return rc;
        return halo(s);
    }
    const bool on_side = sched == 1, serial = sched == 2;
    hipStream_t bs = on_side ? g.side : s;
    if (on_side) {
        IGG_HIP(hipEventRecord(g.ev_fork, s));
        IGG_HIP(hipStreamWaitEvent(g.side, g.ev_fork, 0));
    }
    if ((rc = test_delay(1, on_side ? g.side : s))) return rc;
    if (bnd.nb) {
        if ((rc = timing_mark(bs, 1))) return rc;
        for (int r = 0; r < g.nranks; ++r)
            if ((rc = boundary(r, bnd, bs))) return rc;
        if ((rc = timing_mark(bs, 1))) return rc;
    }
    if (serial) {
        if ((rc = test_delay(3, s))) return rc;
        if ((rc = halo(s))) return rc;
    } else {
        if (!on_side) {
            IGG_HIP(hipEventRecord(g.ev_fork, s));
            IGG_HIP(hipStreamWaitEvent(g.side, g.ev_fork, 0));
        }
        if ((rc = test_delay(3, g.side))) return rc;
        if ((rc = halo(g.side))) return rc;
        IGG_HIP(hipEventRecord(g.ev_join, g.side));
    }
    if ((rc = test_delay(2, s))) return rc;
    for (int r = 0; r < g.nranks && box_points(inner) > 0; ++r) {
        if ((rc = timing_mark(s, 0))) return rc;
        if ((rc = inner_launch(r, inner, s))) return rc;
        if ((rc = timing_mark(s, 0))) return rc;
        if (g.timing) { g.t_launches++; g.t_points += box_points(inner); }
    }
    if (!serial) IGG_HIP(hipStreamWaitEvent(s, g.ev_join, 0));
    return IGG_OK;
}

// One rank that is its own neighbour in every dimension, with the x
// exchange in the stores and the y/z halo filled without send buffers
// (IGG_SLAB_PACK=2).
static bool self_halo_ok()
{
    const Grid &g = grid();
    return g.nranks == 1 && g.fuse_x && g.slab_pack == 2 && g.periods[0] && g.periods[1] && g.periods[2];
}

// The step's launch arguments for rank r: its arrays, the fused x exchange
// into its x neighbours' arrays, and its origin in the global index space.
static int step_args(int r, const igg_field *T2, const igg_field *T, const igg_field *Ci, double lam,
                     double dt, double dx, double dy, double dz, uint32_t key, int stochastic, StepArgs &a)
{
    Grid &g = grid();
    int c[3];
    rank_coords(r, c);
    XHalo xh{0, 0, g.ol[0] - 1, g.n[0] - g.ol[0], 0, 0};
    if (g.fuse_x) {
        const int64_t esz = elem_bytes(T2[r].dtype);
        for (int side = 0; side < 2; ++side) {
            const int q = rank_neighbor(r, 0, side);
            if (q < 0) continue;
            const int64_t diff = (int64_t)((intptr_t)T2[q].data - (intptr_t)T2[r].data);
            if (diff % esz) return fail(IGG_ERR_ARG, "T2 blocks must be aligned to their element size");
            (side == 0 ? xh.on_lo : xh.on_hi) = 1;
            (side == 0 ? xh.d_lo : xh.d_hi) = diff / esz;
        }
    }
    // global indices wrap at the period of a periodic dimension (a point and
    // its copies in overlapping planes draw the same random bits)
    int per[3];
    for (int d = 0; d < 3; ++d) per[d] = g.periods[d] ? g.dims[d] * (g.n[d] - g.ol[d]) : 0;
    const int gnx = g.dims[0] * (g.n[0] - g.ol[0]) + g.ol[0];
    const SrOrigin so{c[0] * (g.n[0] - g.ol[0]), c[1] * (g.n[1] - g.ol[1]), c[2] * (g.n[2] - g.ol[2]),
                      gnx, per[0], per[1], per[2], (gnx + 1) / 2};
    a = StepArgs{T2[r].data, T[r].data, Ci[r].data, g.n[0], g.n[1], g.n[2],
                 dt * lam, 1.0 / (dx * dx), 1.0 / (dy * dy), 1.0 / (dz * dz), key, stochastic, xh, so};
    return IGG_OK;
}

// The slabs and the inner region of one step in one launch (schedule 3).
struct FusedStep {
    int dtype;
    const StepArgs *args;
    const SlabPack *pk;
};
static int fused_step(int r, const Split &slabs, const Box &inner, hipStream_t s, void *ctx)
{
    const FusedStep &f = *static_cast<const FusedStep *>(ctx);
    return launch_step_inner(f.dtype, f.args[r], inner, s, &slabs, f.pk);
}

// diffusion_step for the grid's nranks ranks: fields[r] is rank r's block.
static int step_ranks(const igg_field *T2, const igg_field *T, const igg_field *Ci, double lam, double dt,
                      double dx, double dy, double dz, const int split[3], const igg_rounding *rnd,
                      void *stream)
{
    Grid &g = grid();
    int rc;
    const int P = g.nranks;
    for (int r = 0; r < P; ++r) {
        const std::string sfx = P > 1 ? "[" + std::to_string(r) + "]" : "";
        if ((rc = check_field(&T2[r], ("T2" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&T[r], ("T" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&Ci[r], ("Ci" + sfx).c_str(), true))) return rc;
        if (T2[r].dtype != T[0].dtype || T[r].dtype != T[0].dtype || Ci[r].dtype != T[0].dtype)
            return fail(IGG_ERR_DTYPE, "T2, T and Ci must share one dtype");
    }
    for (int r = 0; r < P; ++r)
        for (int q = 0; q < P; ++q) {
            if (overlaps_mem(T2[r], T[q]) || overlaps_mem(T2[r], Ci[q]))
                return fail(IGG_ERR_ALIAS, "T2 shares memory with T or Ci");
            if (q != r && overlaps_mem(T2[r], T2[q])) return fail(IGG_ERR_ALIAS, "two T2 blocks share memory");
        }
    if ((rc = check_spacings(lam, dt, dx, dy, dz))) return rc;
    if ((rc = check_split(split, g.ol))) return rc;
    int stochastic = 0;
    uint32_t key = 0;
    if (rnd) {
        if (rnd->reserved != 0) return fail(IGG_ERR_ARG, "rounding.reserved must be 0");
        if (rnd->mode != IGG_ROUND_NEAREST && rnd->mode != IGG_ROUND_STOCHASTIC)
            return fail(IGG_ERR_ARG, "unknown rounding mode");
        stochastic = rnd->mode == IGG_ROUND_STOCHASTIC;
        key = sr_key(rnd->seed, rnd->counter);
    }
    std::vector<StepArgs> args(P);
    for (int r = 0; r < P; ++r)
        if ((rc = step_args(r, T2, T, Ci, lam, dt, dx, dy, dz, key, stochastic, args[r]))) return rc;
    if ((rc = ensure_device())) return rc;

    // With x periodic the step kernels also store the x halo of T2 (the
    // exchange between x neighbours on this device is a copy of the two
    // source columns, fused into the kernels that compute them); the halo
    // update then moves the y and z planes only.
    const int halo_dims = g.fuse_x ? 6 : 7;
    const int dtype = T[0].dtype;
    hipStream_t s = (hipStream_t)stream;
    if (!split) {
        Box all{1, g.n[0] - 1, 1, g.n[1] - 1, 1, g.n[2] - 1};
        for (int r = 0; r < P; ++r) {
            if ((rc = timing_mark(s, 0))) return rc;
            if ((rc = launch_step_inner(dtype, args[r], all, s))) return rc;
            if ((rc = timing_mark(s, 0))) return rc;
            if (g.timing) { g.t_launches++; g.t_points += box_points(all); }
        }
        return launch_halo(T2, 1, s, halo_dims);
    }
    // One rank, periodic in every dimension, x exchange in the stores: the
    // slab kernel packs the y and z planes as it computes them, and the
    // exchange and unpack are one copy into the halo planes.
    if (P == 1 && g.fuse_x && g.slab_pack && g.periods[0] && g.periods[1] && g.periods[2]) {
        SlabPack pk{};
        for (int d = 0; d < 2; ++d)
            for (int side = 0; side < 2; ++side) pk.send[d][side] = halo_send_plane(0, d, side);
        for (int d = 0; d < 3; ++d) pk.ol[d] = g.ol[d];
        pk.direct = g.slab_pack == 2;
        FusedStep ctx{dtype, args.data(), &pk};
        return run_split(
            split, dtype,
            [&](hipStream_t st) { return pk.direct ? IGG_OK : launch_unpack_self(T2[0], pk, st); },
            [&](int r, const Split &b, hipStream_t st) { return launch_step_slabs(dtype, args[r], b, &pk, st); },
            [&](int r, const Box &b, hipStream_t st) { return launch_step_inner(dtype, args[r], b, st); }, s, true,
            fused_step, &ctx);
    }
    return run_split(
        split, dtype, [&](hipStream_t st) { return launch_halo(T2, 1, st, halo_dims); },
        [&](int r, const Split &b, hipStream_t st) { return launch_step_boundary(dtype, args[r], b, st); },
        [&](int r, const Box &b, hipStream_t st) { return launch_step_inner(dtype, args[r], b, st); }, s);
}

// update_halo over the grid's ranks: fields[r * nfields + f] is field f of
// rank r; field f has one size and dtype on every rank.
static int update_halo_ranks(const igg_field *fields, int nfields, void *stream)
{
    Grid &g = grid();
    if (!fields) return fail(IGG_ERR_ARG, "fields is null");
    if (nfields < 1 || nfields > IGG_MAX_FIELDS)
        return fail(IGG_ERR_ARG, "nfields must be in 1.." + std::to_string(IGG_MAX_FIELDS));
    int rc;
    const int total = nfields * g.nranks;
    for (int e = 0; e < total; ++e) {
        const int r = e / nfields, f = e % nfields;
        std::string nm = "field " + std::to_string(f) + (g.nranks > 1 ? " of rank " + std::to_string(r) : "");
        if ((rc = check_field(&fields[e], nm.c_str(), false))) return rc;
        const igg_field &f0 = fields[f];
        if (fields[e].dtype != f0.dtype || fields[e].size[0] != f0.size[0] || fields[e].size[1] != f0.size[1] ||
            fields[e].size[2] != f0.size[2])
            return fail(IGG_ERR_SIZE, nm + " differs in size or dtype from the same field of rank 0");
        for (int q = 0; q < e; ++q)
            if (overlaps_mem(fields[e], fields[q]))
                return fail(IGG_ERR_ALIAS, "fields " + std::to_string(q) + " and " + std::to_string(e) +
                                               " share memory");
    }
    if ((rc = ensure_device())) return rc;
    return launch_halo(fields, nfields, (hipStream_t)stream);
}

// The adjoint step of either form (0: Laplacian, 1: staggered flux form)
// for the grid's nranks ranks: each argument is an array of one field per
// rank (a single field on a one-rank grid).
static int adjoint_step(int form, const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                        const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx, double dy,
                        double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    int rc;
    const int P = g.nranks;
    if (!lam_n || !lam_np1 || !T_n || !Ci || !gCi) return fail(IGG_ERR_ARG, "null field");
    const int dt_ = lam_n[0].dtype;
    for (int r = 0; r < P; ++r) {
        const std::string sfx = P > 1 ? "[" + std::to_string(r) + "]" : "";
        if ((rc = check_field(&lam_n[r], ("lam_n" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&lam_np1[r], ("lam_np1" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&T_n[r], ("T_n" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&Ci[r], ("Ci" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&gCi[r], ("gCi" + sfx).c_str(), true))) return rc;
        if (lam_n[r].dtype != dt_ || lam_np1[r].dtype != dt_ || T_n[r].dtype != dt_ || Ci[r].dtype != dt_ ||
            gCi[r].dtype != dt_)
            return fail(IGG_ERR_DTYPE, "adjoint fields must share one dtype");
    }
    if (dt_ == IGG_F16) return fail(IGG_ERR_DTYPE, "the adjoint runs in FP64 or FP32");
    for (int r = 0; r < P; ++r)
        for (int q = 0; q < P; ++q) {
            for (const igg_field *o : {&lam_n[r], &gCi[r]})
                for (const igg_field *i : {&lam_np1[q], &T_n[q], &Ci[q]})
                    if (overlaps_mem(*o, *i)) return fail(IGG_ERR_ALIAS, "an output shares memory with an input");
            if (overlaps_mem(lam_n[r], gCi[q])) return fail(IGG_ERR_ALIAS, "lam_n shares memory with gCi");
            if (q != r && (overlaps_mem(lam_n[r], lam_n[q]) || overlaps_mem(gCi[r], gCi[q])))
                return fail(IGG_ERR_ALIAS, "two ranks' outputs share memory");
        }
    if ((rc = check_spacings(lam, dt, dx, dy, dz))) return rc;
    if ((rc = check_split(split, g.ol))) return rc;
    // per rank: the x exchange of lam_n stored by the adjoint kernels into
    // the x neighbours' lam_n, as in the step
    std::vector<AdjArgs> args(P);
    const int64_t esz = elem_bytes(dt_);
    for (int r = 0; r < P; ++r) {
        XHalo xh{0, 0, g.ol[0] - 1, g.n[0] - g.ol[0], 0, 0};
        if (g.fuse_x)
            for (int side = 0; side < 2; ++side) {
                const int q = rank_neighbor(r, 0, side);
                if (q < 0) continue;
                const int64_t diff = (int64_t)((intptr_t)lam_n[q].data - (intptr_t)lam_n[r].data);
                if (diff % esz) return fail(IGG_ERR_ARG, "lam_n blocks must be aligned to their element size");
                (side == 0 ? xh.on_lo : xh.on_hi) = 1;
                (side == 0 ? xh.d_lo : xh.d_hi) = diff / esz;
            }
        args[r] = form == 0 ? AdjArgs{lam_n[r].data, lam_np1[r].data, T_n[r].data, Ci[r].data, gCi[r].data, g.n[0],
                                      g.n[1], g.n[2], dt * lam, 1.0 / (dx * dx), 1.0 / (dy * dy), 1.0 / (dz * dz),
                                      xh}
                            : AdjArgs{lam_n[r].data, lam_np1[r].data, T_n[r].data, Ci[r].data, gCi[r].data, g.n[0],
                                      g.n[1], g.n[2], dt, 1.0 / dx, 1.0 / dy, 1.0 / dz, xh, 1, lam};
    }
    if ((rc = ensure_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int halo_dims = g.fuse_x ? 6 : 7;
    Box all{1, g.n[0] - 1, 1, g.n[1] - 1, 1, g.n[2] - 1};
    if (split && self_halo_ok() && (g.schedule < 0 || g.schedule == 3)) {
        // one rank, periodic in every dimension: one launch over every inner
        // point, which also stores the x halo of lam_n and, for every inner
        // point that is the image of y/z halo points, those points (the
        // adjoint runs its chain serially anyway, so the boundary has nothing
        // to overlap)
        AdjArgs a0 = args[0];
        const bool sized = lam_n[0].size[1] == g.n[1] && lam_n[0].size[2] == g.n[2];
        if (sized) a0.yz = YZImg{1, g.ol[1] - 1, g.n[1] - g.ol[1], g.ol[2] - 1, g.n[2] - g.ol[2], g.n[1], g.n[2]};
        if ((rc = timing_mark(s, 0))) return rc;
        if ((rc = launch_adjoint_inner(dt_, a0, all, s))) return rc;
        if ((rc = timing_mark(s, 0))) return rc;
        if (g.timing) { g.t_launches++; g.t_points += box_points(all); }
        return sized ? IGG_OK : launch_halo_self_yz(lam_n[0], s);
    }
    if (!split) {
        for (int r = 0; r < P; ++r) {
            if ((rc = timing_mark(s, 0))) return rc;
            if ((rc = launch_adjoint_inner(dt_, args[r], all, s))) return rc;
            if ((rc = timing_mark(s, 0))) return rc;
            if (g.timing) { g.t_launches++; g.t_points += box_points(all); }
        }
        return launch_halo(lam_n, 1, s, halo_dims);
    }
    return run_split(
        split, dt_, [&](hipStream_t st) { return launch_halo(lam_n, 1, st, halo_dims); },
        [&](int r, const Split &b, hipStream_t st) { return launch_adjoint_boxes(dt_, args[r], b.boundary, b.nb, st); },
        [&](int r, const Box &b, hipStream_t st) { return launch_adjoint_inner(dt_, args[r], b, st); }, s, false);
}

static int check_face(const igg_field *q, const char *name, int dim)
{
    Grid &g = grid();
    int rc;
    if ((rc = check_field(q, name, false))) return rc;
    for (int d = 0; d < 3; ++d)
        if (q->size[d] != g.n[d] + (d == dim ? 1 : 0))
            return fail(IGG_ERR_SIZE, std::string(name) + " must have n+1 points in its own dimension "
                                                          "and n in the others");
    return IGG_OK;
}


// The fused flux-form step for the grid's nranks ranks: each argument is an
// array of one field per rank (a single field on a one-rank grid).
static int flux_step_ranks(const igg_field *T2, const igg_field *T, const igg_field *Ci, const igg_field *qx,
                           const igg_field *qy, const igg_field *qz, double lam, double dt, double dx, double dy,
                           double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    int rc;
    const int P = g.nranks;
    if (!T2 || !T || !Ci || !qx || !qy || !qz) return fail(IGG_ERR_ARG, "null field");
    const int ty = T[0].dtype;
    for (int r = 0; r < P; ++r) {
        const std::string sfx = P > 1 ? "[" + std::to_string(r) + "]" : "";
        if ((rc = check_field(&T2[r], ("T2" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&T[r], ("T" + sfx).c_str(), true))) return rc;
        if ((rc = check_field(&Ci[r], ("Ci" + sfx).c_str(), true))) return rc;
        if ((rc = check_face(&qx[r], ("qx" + sfx).c_str(), 0))) return rc;
        if ((rc = check_face(&qy[r], ("qy" + sfx).c_str(), 1))) return rc;
        if ((rc = check_face(&qz[r], ("qz" + sfx).c_str(), 2))) return rc;
        for (const igg_field *f : {&T2[r], &T[r], &Ci[r], &qx[r], &qy[r], &qz[r]})
            if (f->dtype != ty) return fail(IGG_ERR_DTYPE, "flux-form fields must share one dtype");
    }
    if (ty == IGG_F16) return fail(IGG_ERR_DTYPE, "the flux form runs in FP64 or FP32");
    for (int r = 0; r < P; ++r) {
        const igg_field *outs[4] = {&T2[r], &qx[r], &qy[r], &qz[r]};
        for (int o = 0; o < 4; ++o)
            for (int q = 0; q < P; ++q) {
                if (overlaps_mem(*outs[o], T[q]) || overlaps_mem(*outs[o], Ci[q]))
                    return fail(IGG_ERR_ALIAS, "an output shares memory with T or Ci");
                const igg_field *others[4] = {&T2[q], &qx[q], &qy[q], &qz[q]};
                for (int p = 0; p < 4; ++p)
                    if ((q != r || p != o) && overlaps_mem(*outs[o], *others[p]))
                        return fail(IGG_ERR_ALIAS, "outputs share memory");
            }
    }
    if ((rc = check_spacings(lam, dt, dx, dy, dz))) return rc;
    // the face fields overlap their neighbours by ol+1 planes in their own
    // dimension, so each split width must cover that many planes
    const int olf[3] = {g.ol[0] + 1, g.ol[1] + 1, g.ol[2] + 1};
    if ((rc = check_split(split, olf))) return rc;
    // per rank: the x exchange of all four fields is stored by the flux pass
    // into the x neighbours' arrays; the halo update then moves y and z
    std::vector<FluxArgs> args(P);
    const int64_t esz = elem_bytes(ty);
    for (int r = 0; r < P; ++r) {
        FluxXH xh{};
        xh.ol = g.ol[0];
        if (g.fuse_x)
            for (int side = 0; side < 2; ++side) {
                const int q = rank_neighbor(r, 0, side);
                if (q < 0) continue;
                const igg_field *mine[4] = {&T2[r], &qx[r], &qy[r], &qz[r]};
                const igg_field *theirs[4] = {&T2[q], &qx[q], &qy[q], &qz[q]};
                for (int a = 0; a < 4; ++a) {
                    const int64_t diff = (int64_t)((intptr_t)theirs[a]->data - (intptr_t)mine[a]->data);
                    if (diff % esz) return fail(IGG_ERR_ARG, "flux-form blocks must be aligned to their element size");
                    (side == 0 ? xh.d_lo : xh.d_hi)[a] = diff / esz;
                }
                (side == 0 ? xh.on_lo : xh.on_hi) = 1;
            }
        args[r] = FluxArgs{qx[r].data, qy[r].data, qz[r].data, T[r].data, T2[r].data, Ci[r].data, g.n[0], g.n[1],
                           g.n[2], lam, dt, 1.0 / dx, 1.0 / dy, 1.0 / dz, ty, xh};
    }
    if ((rc = ensure_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int halo_dims = g.fuse_x ? 6 : 7;
    std::vector<igg_field> hf((size_t)4 * P);
    for (int r = 0; r < P; ++r) {
        hf[4 * r] = T2[r];
        hf[4 * r + 1] = qx[r];
        hf[4 * r + 2] = qy[r];
        hf[4 * r + 3] = qz[r];
    }
    if (!split) {
        Box all{1, g.n[0] - 1, 1, g.n[1] - 1, 1, g.n[2] - 1};
        for (int r = 0; r < P; ++r) {
            if ((rc = timing_mark(s, 0))) return rc;
            if ((rc = launch_flux_inner(ty, args[r], all, s))) return rc;
            if ((rc = timing_mark(s, 0))) return rc;
            if (g.timing) { g.t_launches++; g.t_points += box_points(all); }
        }
        return launch_halo(hf.data(), 4, s, halo_dims);
    }
    return run_split(
        split, ty, [&](hipStream_t st) { return launch_halo(hf.data(), 4, st, halo_dims); },
        [&](int r, const Split &b, hipStream_t st) { return launch_flux_boxes(ty, args[r], b.boundary, b.nb, st); },
        [&](int r, const Box &b, hipStream_t st) { return launch_flux_inner(ty, args[r], b, st); }, s);
}

}  // namespace igg

using namespace igg;

extern "C" {

const char *igg_last_error(void) { return t_last_error.c_str(); }

const char *igg_version(void) { return "igg-mi355x 0.1 (gfx950)"; }

int igg_init_global_grid(int nx, int ny, int nz, const int dims[3], const int periods[3],
                         const int overlaps[3], int *me)
{
    Grid &g = grid();
    if (g.init) return fail(IGG_ERR_STATE, "the global grid is already initialised");
    int n[3] = {nx, ny, nz};
    int ol[3] = {2, 2, 2}, per[3] = {0, 0, 0}, dm[3] = {1, 1, 1};
    for (int d = 0; d < 3; ++d) {
        if (overlaps) ol[d] = overlaps[d];
        if (periods) per[d] = periods[d];
        if (dims) dm[d] = dims[d] == 0 ? 1 : dims[d];
        if (ol[d] < 2) return fail(IGG_ERR_ARG, "overlaps must be >= 2");
        if (per[d] != 0 && per[d] != 1) return fail(IGG_ERR_ARG, "periods must be 0 or 1");
        if (dm[d] < 0) return fail(IGG_ERR_ARG, "dims must be >= 0");
        if (n[d] < ol[d] + 1)
            return fail(IGG_ERR_ARG, "local size " + std::to_string(n[d]) +
                                         " must exceed the overlap " + std::to_string(ol[d]));
        if (n[d] > (1 << 24)) return fail(IGG_ERR_ARG, "local size above 2^24");
    }
    const int64_t P = (int64_t)dm[0] * dm[1] * dm[2];
    if (P < 1 || P > IGG_MAX_RANKS)
        return fail(IGG_ERR_ARG, "dims must multiply to a rank count in 1.." + std::to_string(IGG_MAX_RANKS));
    if ((int64_t)(nx + 1) * (ny + 1) > 0x7fffffffLL || (int64_t)(nx + 1) * (nz + 1) > 0x7fffffffLL ||
        (int64_t)(ny + 1) * (nz + 1) > 0x7fffffffLL)
        return fail(IGG_ERR_ARG, "a plane of the grid exceeds 2^31 points");
    for (int d = 0; d < 3; ++d) {
        g.n[d] = n[d];
        g.ol[d] = ol[d];
        g.periods[d] = per[d];
        g.dims[d] = dm[d];
    }
    g.nranks = (int)P;
    g.init = true;
    g.timing = false;
    {
        const char *e = getenv("IGG_SCHEDULE");
        const int sv = (e && *e) ? atoi(e) : -1;
        g.schedule = (sv >= 0 && sv <= 3) ? sv : -1;  // anything else: chosen by size and type
        const char *x = getenv("IGG_X_EXCHANGE");
        g.fuse_x = !(x && strcmp(x, "halo") == 0);
        // IGG_TEST_DELAY=<where>:<rounds>, where = side (before the helper
        // stream's first launch), inner (before the inner launch) or halo
        // (before the halo update); rounds of about 3.4 us each, at most 4096
        g.delay_where = 0;
        g.delay_iters = 0;
        const char *td = getenv("IGG_TEST_DELAY");
        if (td && *td) {
            const char *c = strchr(td, ':');
            const size_t len = c ? (size_t)(c - td) : strlen(td);
            int where = 0;
            if (len == 4 && strncmp(td, "side", 4) == 0) where = 1;
            if (len == 5 && strncmp(td, "inner", 5) == 0) where = 2;
            if (len == 4 && strncmp(td, "halo", 4) == 0) where = 3;
            const int it = c ? atoi(c + 1) : 0;
            if (where && it > 0) {
                g.delay_where = where;
                g.delay_iters = std::min(it, 4096);
            }
        }
        const char *sp = getenv("IGG_SLAB_PACK");
        const int spv = (sp && *sp) ? atoi(sp) : -1;
        g.slab_pack = (spv >= 0 && spv <= 2) ? spv : 2;
        const char *zm = getenv("IGG_ZMARCH_MIN_POINTS");
        g.zmarch_min = (zm && *zm) ? atoll(zm) : kZmarchMinPoints;
    }
    g.tev_used = 0;
    g.t_launches = g.t_points = 0;
    if (me) *me = 0;
    return IGG_OK;
}

int igg_global_size(int64_t n_g[3])
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (!n_g) return fail(IGG_ERR_ARG, "n_g is null");
    for (int d = 0; d < 3; ++d)
        n_g[d] = (int64_t)g.dims[d] * (g.n[d] - g.ol[d]) + (int64_t)g.ol[d] * (1 - g.periods[d]);
    return IGG_OK;
}

int igg_topology(int n[3], int dims[3], int periods[3], int overlaps[3], int coords[3])
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    for (int d = 0; d < 3; ++d) {
        if (n) n[d] = g.n[d];
        if (dims) dims[d] = g.dims[d];
        if (periods) periods[d] = g.periods[d];
        if (overlaps) overlaps[d] = g.ol[d];
        if (coords) coords[d] = 0;
    }
    return IGG_OK;
}

int igg_update_halo(const igg_field *fields, int nfields, void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (g.nranks > 1) return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: use igg_update_halo_ranks");
    return update_halo_ranks(fields, nfields, stream);
}

int igg_update_halo_ranks(const igg_field *fields, int nfields, void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    return update_halo_ranks(fields, nfields, stream);
}

int igg_nranks(int *nranks)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (!nranks) return fail(IGG_ERR_ARG, "nranks is null");
    *nranks = g.nranks;
    return IGG_OK;
}

int igg_rank_coords(int rank, int coords[3])
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (!coords) return fail(IGG_ERR_ARG, "coords is null");
    if (rank < 0 || rank >= g.nranks) return fail(IGG_ERR_ARG, "rank out of range");
    rank_coords(rank, coords);
    return IGG_OK;
}

int igg_neighbors(int rank, int lower[3], int upper[3])
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (!lower || !upper) return fail(IGG_ERR_ARG, "null argument");
    if (rank < 0 || rank >= g.nranks) return fail(IGG_ERR_ARG, "rank out of range");
    for (int d = 0; d < 3; ++d) {
        lower[d] = rank_neighbor(rank, d, 0);
        upper[d] = rank_neighbor(rank, d, 1);
    }
    return IGG_OK;
}


int igg_finalize_global_grid(void)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    int rc = release_device();
    g = Grid();
    return rc;
}

int igg_plan_split(const int n[3], const int split[3], int boxes[7][6], int *nboxes)
{
    if (!n || !split || !boxes || !nboxes) return fail(IGG_ERR_ARG, "null argument");
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 3) return fail(IGG_ERR_ARG, "n must be >= 3");
        if (split[d] < 1) return fail(IGG_ERR_ARG, "split widths must be >= 1");
    }
    Split s;
    plan_split(n, split, s);
    for (int q = 0; q < s.nb; ++q) {
        const Box &b = s.boundary[q];
        int v[6] = {b.i0, b.i1, b.j0, b.j1, b.k0, b.k1};
        memcpy(boxes[q], v, sizeof v);
    }
    const Box &b = s.inner;
    int v[6] = {b.i0, b.i1, b.j0, b.j1, b.k0, b.k1};
    memcpy(boxes[s.nb], v, sizeof v);
    *nboxes = s.nb + 1;
    return IGG_OK;
}

int diffusion_step(const igg_field *T2, const igg_field *T, const igg_field *Ci, double lam,
                   double dt, double dx, double dy, double dz, const int split[3],
                   const igg_rounding *rnd, void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (g.nranks > 1) return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: use diffusion_step_ranks");
    if (!T2 || !T || !Ci) return fail(IGG_ERR_ARG, "null field");
    return step_ranks(T2, T, Ci, lam, dt, dx, dy, dz, split, rnd, stream);
}

int diffusion_step_ranks(const igg_field *T2, const igg_field *T, const igg_field *Ci, double lam,
                         double dt, double dx, double dy, double dz, const int split[3],
                         const igg_rounding *rnd, void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (!T2 || !T || !Ci) return fail(IGG_ERR_ARG, "null field array");
    return step_ranks(T2, T, Ci, lam, dt, dx, dy, dz, split, rnd, stream);
}

int diffusion_run(const igg_field *T, const igg_field *T2, const igg_field *Ci, double lam, double dt,
                  double dx, double dy, double dz, const int split[3], const igg_rounding *rnd, int nt,
                  int use_graph, int *final_buf, void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (g.nranks > 1) return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: use diffusion_step_ranks");
    if (!T || !T2 || !Ci || !final_buf) return fail(IGG_ERR_ARG, "null argument");
    if (nt < 0) return fail(IGG_ERR_ARG, "nt must be >= 0");
    if (use_graph && rnd && rnd->mode == IGG_ROUND_STOCHASTIC)
        return fail(IGG_ERR_ARG, "graph replays would repeat the stochastic-rounding counter: use_graph = 0");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    *final_buf = 0;
    const igg_field *buf[2] = {T, T2};
    auto eager = [&](int it) {
        igg_rounding r{};
        const igg_rounding *rp = nullptr;
        if (rnd) {
            r = *rnd;
            r.counter += (uint64_t)it;
            rp = &r;
        }
        const int src = it & 1;
        return step_ranks(buf[1 - src], buf[src], Ci, lam, dt, dx, dy, dz, split, rp, stream);
    };
    if (!use_graph || nt < 2) {
        for (int it = 0; it < nt; ++it)
            if ((rc = eager(it))) return rc;
        *final_buf = nt & 1;
        return IGG_OK;
    }
    // the graph holds `pairs` pairs of steps T -> T2 -> T with these exact
    // arguments (up to 8: one graph launch then covers 16 steps)
    const int pairs = std::min(8, nt / 2);
    std::vector<unsigned char> key;
    auto put = [&](const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        key.insert(key.end(), c, c + n);
    };
    for (const igg_field *f : {T, T2, Ci}) put(f, sizeof(igg_field));
    for (double v : {lam, dt, dx, dy, dz}) put(&v, sizeof v);
    const int nosplit[3] = {-1, -1, -1};
    put(split ? split : nosplit, 3 * sizeof(int));
    const int mode = rnd ? rnd->mode : -1;
    put(&mode, sizeof mode);
    put(&pairs, sizeof pairs);
    if (!g.run_exec || key != g.run_key) {
        // a new argument set is captured: both steps run their argument
        // checks while being recorded, and a failed check ends the capture
        // without keeping anything
        if ((rc = ensure_device())) return rc;
        if (!g.cap) IGG_HIP(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
        if (g.run_exec) {
            IGG_HIP(hipGraphExecDestroy(g.run_exec));
            g.run_exec = nullptr;
            g.run_key.clear();
        }
        const bool timing = g.timing;
        g.timing = false;
        IGG_HIP(hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal));
        int rc2 = IGG_OK;
        for (int p = 0; p < pairs && !rc2; ++p) {
            rc2 = step_ranks(T2, T, Ci, lam, dt, dx, dy, dz, split, rnd, g.cap);
            if (!rc2) rc2 = step_ranks(T, T2, Ci, lam, dt, dx, dy, dz, split, rnd, g.cap);
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(g.cap, &graph);
        g.timing = timing;
        if (rc2) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc2;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        g.run_exec = exec;
        g.run_key = key;
    }
    const int replays = nt / (2 * pairs);
    for (int p = 0; p < replays; ++p) IGG_HIP(hipGraphLaunch(g.run_exec, s));
    for (int it = replays * 2 * pairs; it < nt; ++it)
        if ((rc = eager(it))) return rc;
    *final_buf = nt & 1;
    return IGG_OK;
}

int diffusion_dt(const igg_field *Ci, double lam, double dx, double dy, double dz, double *dt,
                 void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    int rc;
    if ((rc = check_field(Ci, "Ci", false))) return rc;
    if (!dt) return fail(IGG_ERR_ARG, "dt is null");
    if ((rc = check_spacings(lam, 0.0, dx, dy, dz))) return rc;
    if ((rc = ensure_device())) return rc;
    double m = 0.0;
    if ((rc = launch_reduce(IGG_RED_MAX, *Ci, nullptr, &m, (hipStream_t)stream))) return rc;
    if (!(m > 0.0) || !isfinite(m)) return fail(IGG_ERR_ARG, "maximum(Ci) must be positive and finite");
    double mn = std::min(dx * dx, std::min(dy * dy, dz * dz));
    *dt = mn / lam / m / 6.1;
    return IGG_OK;
}

int diffusion_step_adjoint(const igg_field *lam_n, const igg_field *lam_np1,
                           const igg_field *T_n, const igg_field *Ci, const igg_field *gCi,
                           double lam, double dt, double dx, double dy, double dz,
                           const int split[3], void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (g.nranks > 1)
        return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: use diffusion_step_adjoint_ranks");
    return adjoint_step(0, lam_n, lam_np1, T_n, Ci, gCi, lam, dt, dx, dy, dz, split, stream);
}

int diffusion_step_adjoint_ranks(const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                                 const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx,
                                 double dy, double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    return adjoint_step(0, lam_n, lam_np1, T_n, Ci, gCi, lam, dt, dx, dy, dz, split, stream);
}


int diffusion_flux_step(const igg_field *T2, const igg_field *T, const igg_field *Ci,
                        const igg_field *qx, const igg_field *qy, const igg_field *qz, double lam,
                        double dt, double dx, double dy, double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (g.nranks > 1) return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: use diffusion_flux_step_ranks");
    return flux_step_ranks(T2, T, Ci, qx, qy, qz, lam, dt, dx, dy, dz, split, stream);
}

int diffusion_flux_step_ranks(const igg_field *T2, const igg_field *T, const igg_field *Ci,
                              const igg_field *qx, const igg_field *qy, const igg_field *qz, double lam,
                              double dt, double dx, double dy, double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    return flux_step_ranks(T2, T, Ci, qx, qy, qz, lam, dt, dx, dy, dz, split, stream);
}

int diffusion_flux_step_adjoint(const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                                const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx,
                                double dy, double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (g.nranks > 1)
        return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: use diffusion_flux_step_adjoint_ranks");
    return adjoint_step(1, lam_n, lam_np1, T_n, Ci, gCi, lam, dt, dx, dy, dz, split, stream);
}

int diffusion_flux_step_adjoint_ranks(const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                                      const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx,
                                      double dy, double dz, const int split[3], void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    return adjoint_step(1, lam_n, lam_np1, T_n, Ci, gCi, lam, dt, dx, dy, dz, split, stream);
}

// Argument checks of igg_reduce and igg_reduce_noalloc (host only); *two is
// set when the operation reads b.
static int check_reduce(int op, const igg_field *a, const igg_field *b, const double *out, bool *two)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    if (!out) return fail(IGG_ERR_ARG, "out is null");
    if (op < IGG_RED_MAX || op > IGG_RED_MAX_ABS) return fail(IGG_ERR_ARG, "unknown reduction");
    int rc;
    if ((rc = check_field(a, "a", false))) return rc;
    *two = op == IGG_RED_SUM_RATIO || op == IGG_RED_HALF_SQDIFF || op == IGG_RED_DOT || op == IGG_RED_MAX_ABS_DIFF;
    if (*two) {
        if ((rc = check_field(b, "b", false))) return rc;
        for (int d = 0; d < 3; ++d)
            if (a->size[d] != b->size[d]) return fail(IGG_ERR_SIZE, "a and b differ in size");
        if (a->dtype != b->dtype) return fail(IGG_ERR_DTYPE, "a and b must share one dtype");
    }
    return IGG_OK;
}

int igg_reduce(int op, const igg_field *a, const igg_field *b, double *out, void *stream)
{
    bool two = false;
    int rc;
    if ((rc = check_reduce(op, a, b, out, &two))) return rc;
    if ((rc = ensure_device())) return rc;
    return launch_reduce(op, *a, two ? b : nullptr, out, (hipStream_t)stream);
}

int igg_adjoint_seed(const igg_field *T, const igg_field *T_obs, const igg_field *lam, int halo, double *loss,
                     void *stream)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    int rc;
    if ((rc = check_field(lam, "lam", true))) return rc;
    if (T_obs && !T) return fail(IGG_ERR_ARG, "T_obs without T");
    if (loss && !T_obs) return fail(IGG_ERR_ARG, "the loss needs T and T_obs");
    if (halo != 0 && halo != 1) return fail(IGG_ERR_ARG, "halo must be 0 or 1");
    if (halo && g.nranks > 1)
        return fail(IGG_ERR_STATE, "the grid holds several virtual ranks: seed each block with halo = 0, then "
                                   "igg_update_halo_ranks");
    for (const igg_field *f : {T, T_obs}) {
        if (!f) continue;
        if ((rc = check_field(f, f == T ? "T" : "T_obs", true))) return rc;
        if (f->dtype != lam->dtype) return fail(IGG_ERR_DTYPE, "T, T_obs and lam must share one dtype");
        if (overlaps_mem(*f, *lam)) return fail(IGG_ERR_ALIAS, "lam shares memory with an input");
    }
    if ((rc = ensure_device())) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = launch_seed(T, T_obs, *lam, loss, s))) return rc;
    if (halo && (rc = launch_halo(lam, 1, s))) return rc;
    return loss ? read_reduce_result(loss, s) : IGG_OK;
}

int igg_reduce_noalloc(int op, const igg_field *a, const igg_field *b, double *out_dev, void *stream)
{
    bool two = false;
    int rc;
    if ((rc = check_reduce(op, a, b, out_dev, &two))) return rc;
    return launch_reduce_noalloc(op, *a, two ? b : nullptr, out_dev, (hipStream_t)stream);
}

int igg_timing_enable(int on)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    g.timing = on != 0;
    if (g.timing) {
        // make the event pool now, so that timed work does not pay for
        // creating events (it grows later if more launches are timed)
        int rc;
        if ((rc = ensure_device())) return rc;
        while (g.tev.size() < kTimingPool) {
            hipEvent_t e;
            IGG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            g.tev.push_back(e);
            g.tev_kind.push_back(0);
        }
    }
    return IGG_OK;
}

int igg_timing_read(double *ms, int64_t *launches, int64_t *points, double *boundary_ms)
{
    Grid &g = grid();
    if (!g.init) return fail(IGG_ERR_STATE, "the global grid is not initialised");
    double total[2] = {0.0, 0.0};
    for (size_t q = 0; q + 1 < g.tev_used; q += 2) {
        float t = 0.f;
        IGG_HIP(hipEventSynchronize(g.tev[q + 1]));
        IGG_HIP(hipEventElapsedTime(&t, g.tev[q], g.tev[q + 1]));
        total[g.tev_kind[q] ? 1 : 0] += t;
    }
    if (ms) *ms = total[0];
    if (boundary_ms) *boundary_ms = total[1];
    if (launches) *launches = g.t_launches;
    if (points) *points = g.t_points;
    g.tev_used = 0;
    g.t_launches = g.t_points = 0;
    return IGG_OK;
}

}  // extern "C"
