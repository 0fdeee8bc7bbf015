// host.hpp -- host-side state of the implicit global grid and the launchers
// each kernel file provides to the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include <algorithm>

#include "igg.h"
#include "device.hpp"

namespace igg {

// ------------------------------------------------------------------ errors
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define IGG_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::igg::hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------ launch shapes
inline int64_t box_count(const Box &b)
{
    return (int64_t)std::max(0, b.i1 - b.i0) * std::max(0, b.j1 - b.j0) * std::max(0, b.k1 - b.k0);
}

// Regions below zmarch_min_points() points (default 2^21) go to the
// one-thread-per-point box kernels: their z-march tiles would be too few to
// fill the chip, and such fields sit in the caches anyway.
constexpr int64_t kZmarchMinPoints = (int64_t)1 << 21;
int64_t zmarch_min_points();

// Planes per z-march work-group: the largest of zc_max, zc_max/2, ... (at
// least 4) that still gives `target` work-groups for `columns` tiles over
// `depth` planes.  More, shorter marches balance the compute units better;
// the planes two chunks share are read at about the same time, mostly from
// cache, so short chunks add little traffic.
inline int zchunk_for_groups(int64_t columns, int depth, int zc_max, int64_t target = 2048)
{
    int zc = zc_max;
    while (zc > 4 && columns * ((depth + zc - 1) / zc) < target) zc /= 2;
    return zc < 1 ? 1 : zc;
}

// ------------------------------------------------------------------ state
// The one implicit global grid of the process (the paper's calls take no
// handle).  Device resources are created on first GPU use.
struct Grid {
    bool init = false;
    int n[3] = {0, 0, 0};
    int dims[3] = {1, 1, 1};
    int periods[3] = {0, 0, 0};
    int ol[3] = {2, 2, 2};

    bool dev_ready = false;
    int device = -1;
    hipStream_t side = nullptr;       // helper stream: boundary slabs + halo chain
    hipEvent_t ev_fork = nullptr;     // caller stream -> helper stream
    hipEvent_t ev_join = nullptr;     // helper stream -> caller stream

    int nranks = 1;                     // virtual ranks held by this process (product of dims)
    unsigned char *halo_buf = nullptr;  // send and receive planes of every rank
    size_t halo_cap = 0;                // bytes of one side of one field (one plane)

    double *red_part = nullptr;  // per-block partial results
    double *red_host = nullptr;  // pinned host result

    int schedule = -1;  // 1: slabs + update on the helper stream, 0: slabs first on the caller
                        // stream, 2: one chain on the caller stream, -1: 1 or 2 by size
    int fuse_x = 1;    // x exchange fused into the step kernels' stores
    int slab_pack = 2;  // y/z halo planes packed by the boundary-slab kernel (one periodic rank):
                        // 0 separate halo pass, 1 send planes + one unpack copy, 2 into the halo planes
    int delay_where = 0, delay_iters = 0;  // IGG_TEST_DELAY: a fixed wait put into one stream
    int64_t zmarch_min = kZmarchMinPoints;  // smallest region for the z-march kernels

    // diffusion_run's graph: two steps T -> T2 -> T captured on the capture
    // stream, kept while every argument the kernels take stays the same
    hipStream_t cap = nullptr;
    hipGraphExec_t run_exec = nullptr;
    std::vector<unsigned char> run_key;

    bool timing = false;
    std::vector<hipEvent_t> tev;  // start/stop pairs of timed launches
    std::vector<int> tev_kind;    // 0: inner-region kernel, 1: boundary kernels
    size_t tev_used = 0;
    int64_t t_launches = 0, t_points = 0;
};

Grid &grid();
int ensure_device();  // create stream, events, buffers on the current device

// ------------------------------------------------------------ validation
int check_field(const igg_field *f, const char *name, bool grid_sized);
int64_t field_elems(const igg_field &f);
int elem_bytes(int dtype);
bool overlaps_mem(const igg_field &a, const igg_field &b);

// ------------------------------------------------------------ schedules
struct Split {
    Box boundary[6];
    int kind[6];  // 0: x slab, 1: y or z slab
    int nb = 0;
    Box inner;
};
int plan_split(const int n[3], const int w[3], Split &s);
BoxSet make_boxset(const Box *b, int nb);

// ------------------------------------------------------------ ranks
// Virtual rank r of a dims[0] x dims[1] x dims[2] topology has coordinates
// (r % dims[0], (r / dims[0]) % dims[1], r / (dims[0] * dims[1])).
void rank_coords(int r, int c[3]);
// Neighbour of rank r in dimension d on side s (0 lower, 1 upper), or -1
// at the edge of a non-periodic dimension.
int rank_neighbor(int r, int d, int s);

// ------------------------------------------------------------- launchers
// Halo update of fields (already validated) on `s`: fields[r * nf + f] is
// field f of rank r, for the grid's nranks ranks.
// dims: bit d set = update dimension d (x = bit 0)
int launch_halo(const igg_field *f, int nf, hipStream_t s, int dims = 7);

// x exchange fused into a step kernel.  The point computed at x = lo (ol-1)
// is also stored at x = nx-1 of the lower x neighbour's array (on_lo), the
// point at x = hi (nx-ol) at x = 0 of the upper neighbour's array (on_hi);
// d_lo and d_hi are those arrays' offsets from the own array in elements (0
// when the process is its own neighbour).  That is the x halo update of the
// result, done by the thread that computes the point.
struct XHalo {
    int on_lo, on_hi, lo, hi;
    int64_t d_lo, d_hi;
};

struct StepArgs {
    void *T2;
    const void *T;
    const void *Ci;
    int nx, ny, nz;
    double a, rx, ry, rz;  // dt*lam, 1/dx^2, 1/dy^2, 1/dz^2
    uint32_t key;          // FP16 stochastic-rounding key
    int stochastic;
    XHalo xh;
    SrOrigin so;
};
int launch_step_boxes(int dtype, const StepArgs &a, const Box *b, int nb, hipStream_t s);
struct SlabPack;
// The inner region b; with `slabs`, the y and z slabs of that split (and the
// pack pk) run in the same launch, by its first work-groups.
int launch_step_inner(int dtype, const StepArgs &a, const Box &b, hipStream_t s, const Split *slabs = nullptr,
                      const SlabPack *pk = nullptr);
int launch_step_boundary(int dtype, const StepArgs &a, const Split &sp, hipStream_t s);

// The y and z halo planes of one rank that is its own neighbour in every
// dimension, packed by the boundary-slab kernel as it computes them.
// send[d][s] holds the plane of dimension d+1 (y, then z) sent to the lower
// (s = 0: plane ol-1) or the upper (s = 1: plane n-ol) neighbour, x
// fastest: nx*nz elements (y) or nx*ny (z).  Every entry, the plane's own
// halo rows and columns included, ends up holding the value the
// dimension-ordered halo update leaves at that point of its destination.
struct SlabPack {
    void *send[2][2];
    int ol[3];
    int direct;  // 1: store straight into the halo planes of T2 (no send buffers, no unpack)
};
// The y and z slabs of sp (kind 1) with one wavefront per row run, marching
// along the slab; with pk, the pack of the y and z halo planes fused in.
int launch_step_slabs(int dtype, const StepArgs &a, const Split &sp, const SlabPack *pk, hipStream_t s);
// Exchange and unpack of a SlabPack for the self-neighbour: each packed plane
// is copied into the halo plane of f it fills (y plane side 0 -> j = ny-1,
// side 1 -> j = 0; z likewise), one launch for the four planes.
int launch_unpack_self(const igg_field &f, const SlabPack &pk, hipStream_t s);
// The y and z halo update of f for one rank that is its own neighbour in
// every dimension, in one launch: every point of the y and z halo planes
// takes the value of its image among the inner points, which is what the
// dimension-ordered update leaves there (the x halo columns of inner rows
// must already hold their images; the step kernels store them).
int launch_halo_self_yz(const igg_field &f, hipStream_t s);
// Send buffer of rank r, slot f (a field index of the halo update), side.
unsigned char *halo_send_plane(int r, int f, int side);

// The y and z halo planes of lam_n filled by the adjoint kernels' stores,
// on one rank that is its own neighbour in every dimension: halo row ny-1
// is the image of row jl = ol-1, row 0 that of row jh = ny-ol (z likewise,
// kl and kh), and a point's image has the same x index (its x-halo copies
// come with the x exchange).  Each point of the four planes has one image
// among the inner points, so these stores fill the planes.
struct YZImg {
    int on;
    int jl, jh, kl, kh;
    int ny, nz;
};

struct AdjArgs {
    void *lam_n;
    const void *lp;
    const void *Tn;
    const void *Ci;
    void *gCi;
    int nx, ny, nz;
    double a, rx, ry, rz;  // Laplacian form: dt*lam, 1/dd^2; flux form: dt, 1/dd
    XHalo xh;              // x exchange of lam_n fused into the stores
    int form = 0;          // 0: Laplacian step, 1: staggered flux form
    double lamf = 0.0;     // lam, for the flux form's face fluxes
    YZImg yz{};            // y/z halo of lam_n stored with its images (on: set)
};
int launch_adjoint_boxes(int dtype, const AdjArgs &a, const Box *b, int nb, hipStream_t s);
int launch_adjoint_inner(int dtype, const AdjArgs &a, const Box &b, hipStream_t s);

// x exchange of the four flux-form fields fused into the flux pass: T2, qy
// and qz (nx points in x, overlap ol) send column ol-1 to the lower x
// neighbour's column nx-1 and column nx-ol to the upper neighbour's column
// 0; qx (nx+1 faces, overlap ol+1) sends face ol to the lower neighbour's
// face nx and face nx-ol to the upper neighbour's face 0.  d_lo[a] and
// d_hi[a] are the neighbours' arrays' offsets from the own ones in elements,
// a = T2, qx, qy, qz (0 when the process is its own neighbour).
struct FluxXH {
    int on_lo, on_hi, ol;
    int64_t d_lo[4], d_hi[4];
};

struct FluxArgs {
    void *qx, *qy, *qz;
    const void *T;
    void *T2;
    const void *Ci;
    int nx, ny, nz;
    double lam, dt, rdx, rdy, rdz;
    int dtype;
    FluxXH xh;  // x exchange of T2, qx, qy, qz fused into the stores
};
// The fused flux-form step (faces, update, x exchange) over boxes of cells:
// one thread per cell, or z-march tiles for a large region.
int launch_flux_boxes(int dtype, const FluxArgs &a, const Box *b, int nb, hipStream_t s);
int launch_flux_inner(int dtype, const FluxArgs &a, const Box &b, hipStream_t s);


int launch_reduce(int op, const igg_field &a, const igg_field *b, double *out, hipStream_t s);
// lam = a - b (or a, or 0) on the inner points of lam, zero on its halo;
// with loss, the FP64 loss 0.5*sum (a-b)^2 is left for read_reduce_result.
int launch_seed(const igg_field *a, const igg_field *b, const igg_field &lam, double *loss, hipStream_t s);
// The value the last reduction left on the device, after synchronising s.
int read_reduce_result(double *out, hipStream_t s);
// The same reduction into *out_dev (device memory), with the partial results
// in the library's static device array instead of the grid's buffers: no
// allocation, no synchronisation.
constexpr int IGG_MAX_DEVICES = 64;
int launch_reduce_noalloc(int op, const igg_field &a, const igg_field *b, double *out_dev, hipStream_t s);

// FP16 stochastic-rounding key of a (seed, counter) pair.
uint32_t sr_key(uint64_t seed, uint64_t counter);

}  // namespace igg
