// step.hip -- the explicit diffusion step of Fig. 1 (`step!`) for FP64, FP32
// and FP16 storage.
//
// Two kernels compute points, both through igg::diffuse, so a point's bits
// do not depend on which of them computed it:
//   k_step_boxes   one thread per point over up to six boxes (the y and z
//                  boundary slabs, and any region too small for z-march
//                  tiles); plain global loads.
//   k_step_zmarch  the inner region and the x slabs: each work-group owns a
//                  TW x TH tile of (x, y) columns and marches up a chunk of z
//                  planes.  Every thread keeps T at k-1, k, k+1 (and k+2 in
//                  flight) for its RY rows of VEC points in registers, writes
//                  plane k to a double-buffered LDS tile, and takes its x and
//                  y neighbours from there or from its own registers.  Thread
//                  rows 0 and TY-1 also load the y-halo rows, lanes 0 and
//                  BX-1 the x-halo points.
// Both store the x halo of T2 as they compute the points the x exchange
// moves (XHalo), and hash a point's global index for FP16 stochastic
// rounding (SrOrigin).
#include <stdlib.h>

#include <type_traits>

#include "host.hpp"

namespace igg {

template <typename S, int VEC> struct VecOf {
    typedef S type __attribute__((ext_vector_type(VEC)));
};
template <typename S> struct VecOf<S, 1> {
    typedef S type;
};

template <typename S, int VEC>
__device__ __forceinline__ S lane_elem(const typename VecOf<S, VEC>::type &v, int q)
{
    if constexpr (VEC == 1)
        return v;
    else
        return v[q];
}

// element q of a vector for a q known only at run time
template <typename S, int VEC>
__device__ __forceinline__ S lane_elem_dyn(const typename VecOf<S, VEC>::type &v, int q)
{
    S x = lane_elem<S, VEC>(v, 0);
#pragma unroll
    for (int p = 1; p < VEC; ++p)
        if (q == p) x = lane_elem<S, VEC>(v, p);
    return x;
}

template <typename S, int VEC>
__device__ __forceinline__ void set_elem(typename VecOf<S, VEC>::type &v, int q, S x)
{
    if constexpr (VEC == 1)
        v = x;
    else
        v[q] = x;
}

// --------------------------------------------------------------- boxes
template <typename S>
__global__ void __launch_bounds__(256)
k_step_boxes(S *__restrict__ T2, const S *__restrict__ T, const S *__restrict__ Ci, BoxSet bs, int nx,
             int ny, compute_t<S> a, compute_t<S> rx, compute_t<S> ry, compute_t<S> rz, uint32_t key,
             int stochastic, XHalo xh, SrOrigin so)
{
    using C = compute_t<S>;
    int i, j, k;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!boxset_point(bs, t, i, j, k)) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t p = i + sy * j + sz * k;
    C c = widen<C>(T[p]);
    C out = diffuse<C>(c, widen<C>(T[p - 1]), widen<C>(T[p + 1]), widen<C>(T[p - sy]), widen<C>(T[p + sy]),
                       widen<C>(T[p - sz]), widen<C>(T[p + sz]), widen<C>(Ci[p]), a, rx, ry, rz);
    uint32_t r = 0;
    if (stochastic) r = sr_point_bits(sr_plane_key(key, k, so), i, j, so);
    const S v = Store<S>::put(out, r, stochastic);
    T2[p] = v;
    if (xh.on_lo && i == xh.lo) T2[p - i + nx - 1 + xh.d_lo] = v;
    if (xh.on_hi && i == xh.hi) T2[p - i + xh.d_hi] = v;
}

// ------------------------------------------------------- boundary slabs
// The y and z slabs of the boundary-first step: a few rows thick across one
// dimension (the thin one), whole in x and in the other dimension.  One
// wavefront takes a run of 64*VEC points of one row across its lanes and
// marches along the slab's long in-plane dimension (z for a y slab, y for a
// z slab).  Per point it holds T of the row one step behind, at and one step
// ahead, and of the two neighbour rows across the thin dimension, in
// registers, so each step reads three new rows of T (ahead, and both
// neighbours): the least a slab one row thick can read.  x neighbours come
// from the adjacent lanes by cross-lane shuffles, the two beyond the run's
// ends from memory.  No LDS and no barriers: the waves of a work-group are
// independent.
//
// With `pack` set (one rank, every dimension periodic: the process is its
// own neighbour) the kernel also writes the y and z send planes of the halo
// update as it computes their points: the pack of the update fused into the
// stores, as the x exchange is.  An entry of a send plane that lies in an
// x halo column, or in a halo row of the plane's other dimension, holds the
// image of an inner point (the value the dimension-ordered update would
// leave there), and the thread that computes that point stores it there
// too.  So every entry of a packed plane is final, and the planes can be
// unpacked in any order.  With `direct` packing the planes are the halo
// planes of T2 they fill: the exchange with oneself and the unpack become
// these stores, as for the x exchange.
struct SlabBox {
    Box b;
    int mz;         // 1: march along z (a y slab, rows j); 0: march along y (a z slab, rows k)
    int nxs;        // runs of 64*VEC points per row
    int nrow;       // rows across the thin dimension
    int64_t first;  // first wave of this box
};
struct SlabSet {
    SlabBox s[4];
    int n;
    int mc;  // march steps per chunk
    int64_t waves;
    int nx, ny, nz;
    XHalo xh;
    SrOrigin so;
    int pack;
    void *send[2][2];    // [0]: y planes, [1]: z planes; side 0 goes to the lower neighbour
    int64_t bstride[2];  // elements between consecutive rows of a y / z plane
    int src[2][2];       // plane index packed into send[d][s] (ol-1 and n-ol)
    int img[3][2];     // per dimension: the index whose image is n-1 (ol-1) and 0 (n-ol)
};

template <typename S, int VEC>
__device__ __forceinline__ void slab_put_row(S *row, int i, bool xin, bool full, int i0, int i1,
                                             const typename VecOf<S, VEC>::type &out)
{
    using V = typename VecOf<S, VEC>::type;
    if (full) {
        *reinterpret_cast<V *>(row + i) = out;
    } else if (xin) {
#pragma unroll
        for (int q = 0; q < VEC; ++q)
            if (i + q >= i0 && i + q < i1) row[i + q] = lane_elem<S, VEC>(out, q);
    }
}

// Wave w of the slab work (lane `lane`); waves past the end return.  SR:
// stochastic rounding of FP16 stores (a template argument, so a kernel
// without it carries none of its code).
template <typename S, int VEC, int SR>
__device__ __forceinline__ void slab_body(S *__restrict__ T2, const S *__restrict__ T, const S *__restrict__ Ci,
                                          const SlabSet &ss, compute_t<S> a, compute_t<S> rx, compute_t<S> ry,
                                          compute_t<S> rz, uint32_t key, int64_t w, int lane)
{
    constexpr int stochastic = SR;
    using C = compute_t<S>;
    using V = typename VecOf<S, VEC>::type;
    constexpr int RUN = 64 * VEC;
    if (w >= ss.waves) return;
    int q = 0;
#pragma unroll
    for (int p = 1; p < 4; ++p)
        if (p < ss.n && w >= ss.s[p].first) q = p;
    const Box bb = ss.s[q].b;
    const int mz = ss.s[q].mz, nxs = ss.s[q].nxs, nrow = ss.s[q].nrow;
    int64_t loc = w - ss.s[q].first;
    const int xs = (int)(loc % nxs);
    loc /= nxs;
    const int row = (int)(loc % nrow);
    const int ch = (int)(loc / nrow);

    const int nx = ss.nx, ny = ss.ny;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int x0 = xs * RUN;
    const int i = x0 + lane * VEC;
    const bool xin = i < nx;
    const bool full = xin && i >= bb.i0 && i + VEC <= bb.i1;
    // the row's fixed index across the thin dimension, the march range, and
    // the strides across (st) and along (sm) the march
    const int fixed = mz ? bb.j0 + row : bb.k0 + row;
    const int mlo = mz ? bb.k0 : bb.j0, mhi = mz ? bb.k1 : bb.j1;
    const int m0 = mlo + ch * ss.mc;
    const int m1 = (m0 + ss.mc < mhi) ? m0 + ss.mc : mhi;
    const int64_t st = mz ? sy : sz, sm = mz ? sz : sy;
    int64_t p = mz ? (int64_t)fixed * sy + (int64_t)m0 * sz : (int64_t)m0 * sy + (int64_t)fixed * sz;

    auto ld = [&](int64_t off) -> V {
        V v{};
        if (xin) v = *reinterpret_cast<const V *>(T + off + i);
        return v;
    };
    // Ci is read once per step: non-temporal
    auto ld_ci = [&](int64_t off) -> V {
        V v{};
        if (xin) v = __builtin_nontemporal_load(reinterpret_cast<const V *>(Ci + off + i));
        return v;
    };
    // the x neighbour beyond the run's end: lane 0 holds x0-1, lane 63 x0+RUN
    auto edge = [&](int64_t off) -> C {
        C e = C(0);
        if (lane == 0 && x0 > 0) e = widen<C>(T[off + x0 - 1]);
        if (lane == 63 && x0 + RUN < nx) e = widen<C>(T[off + x0 + RUN]);
        return e;
    };

    V tm = ld(p - sm), tc = ld(p), tp = ld(p + sm);
    V rl = ld(p - st), rh = ld(p + st);
    V ci = ld_ci(p);
    C ec = edge(p);
    for (int m = m0; m < m1; ++m) {
        const bool more = m + 1 < m1;
        V tn{}, rln{}, rhn{}, cn{};
        C en = C(0);
        if (more) {
            tn = ld(p + 2 * sm);
            rln = ld(p + sm - st);
            rhn = ld(p + sm + st);
            cn = ld_ci(p + sm);
            en = edge(p + sm);
        }
        C fromlo = __shfl(widen<C>(lane_elem<S, VEC>(tc, VEC - 1)), lane > 0 ? lane - 1 : 0);
        C fromhi = __shfl(widen<C>(lane_elem<S, VEC>(tc, 0)), lane < 63 ? lane + 1 : 63);
        if (lane == 0) fromlo = ec;
        if (lane == 63) fromhi = ec;
        const int jc = mz ? fixed : m, kc = mz ? m : fixed;
        const uint32_t pk = stochastic ? sr_plane_key(key, kc, ss.so) : 0u;
        uint32_t rbits[VEC];
        if constexpr (SR) {
            if constexpr (VEC % 2 == 0) {
#pragma unroll
                for (int e = 0; e < VEC; e += 2) sr_point_bits2(pk, i + e, jc, ss.so, rbits[e], rbits[e + 1]);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) rbits[e] = sr_point_bits(pk, i + e, jc, ss.so);
            }
        }
        V out;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const C c = widen<C>(lane_elem<S, VEC>(tc, e));
            const C xm = e == 0 ? fromlo : widen<C>(lane_elem<S, VEC>(tc, e - 1));
            const C xp = e == VEC - 1 ? fromhi : widen<C>(lane_elem<S, VEC>(tc, e + 1));
            const C across_m = widen<C>(lane_elem<S, VEC>(rl, e)), across_p = widen<C>(lane_elem<S, VEC>(rh, e));
            const C along_m = widen<C>(lane_elem<S, VEC>(tm, e)), along_p = widen<C>(lane_elem<S, VEC>(tp, e));
            const C ym = mz ? across_m : along_m, yp = mz ? across_p : along_p;
            const C zm = mz ? along_m : across_m, zp = mz ? along_p : across_p;
            const C v = diffuse<C>(c, xm, xp, ym, yp, zm, zp, widen<C>(lane_elem<S, VEC>(ci, e)), a, rx, ry, rz);
            set_elem<S, VEC>(out, e, Store<S>::put(v, stochastic ? rbits[e] : 0u, stochastic));
        }
        S *dst = T2 + p;
        if (full) {
            __builtin_nontemporal_store(out, reinterpret_cast<V *>(dst + i));
        } else if (xin) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (i + e >= bb.i0 && i + e < bb.i1) dst[i + e] = lane_elem<S, VEC>(out, e);
        }
        // the x exchange fused into the stores, as in the other step kernels
        if (ss.xh.on_lo && xin && i <= ss.xh.lo && i + VEC > ss.xh.lo)
            dst[nx - 1 + ss.xh.d_lo] = lane_elem_dyn<S, VEC>(out, ss.xh.lo - i);
        if (ss.xh.on_hi && xin && i <= ss.xh.hi && i + VEC > ss.xh.hi)
            dst[ss.xh.d_hi] = lane_elem_dyn<S, VEC>(out, ss.xh.hi - i);
        if (ss.pack) {
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                // d = 0: y planes (entries x + nx*k), d = 1: z planes (entries x + nx*j)
                const int own = d == 0 ? jc : kc;
                const int b = d == 0 ? kc : jc;
                const int bn = d == 0 ? ss.nz : ny;
                const int bd = d == 0 ? 2 : 1;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if (own != ss.src[d][side]) continue;
                    S *P = reinterpret_cast<S *>(ss.send[d][side]);
                    const int rows[3] = {b, b == ss.img[bd][0] ? bn - 1 : -1, b == ss.img[bd][1] ? 0 : -1};
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        if (rows[r] < 0) continue;
                        S *R = P + ss.bstride[d] * rows[r];
                        slab_put_row<S, VEC>(R, i, xin, full, bb.i0, bb.i1, out);
                        if (xin && i <= ss.img[0][0] && i + VEC > ss.img[0][0])
                            R[nx - 1] = lane_elem_dyn<S, VEC>(out, ss.img[0][0] - i);
                        if (xin && i <= ss.img[0][1] && i + VEC > ss.img[0][1])
                            R[0] = lane_elem_dyn<S, VEC>(out, ss.img[0][1] - i);
                    }
                }
            }
        }
        tm = tc;
        tc = tp;
        tp = tn;
        rl = rln;
        rh = rhn;
        ci = cn;
        ec = en;
        p += sm;
    }
}

template <typename S, int VEC, int SR>
__global__ void __launch_bounds__(256)
k_step_slab(S *__restrict__ T2, const S *__restrict__ T, const S *__restrict__ Ci, SlabSet ss,
            compute_t<S> a, compute_t<S> rx, compute_t<S> ry, compute_t<S> rz, uint32_t key)
{
    slab_body<S, VEC, SR>(T2, T, Ci, ss, a, rx, ry, rz, key,
                          (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), threadIdx.x & 63);
}

// --------------------------------------------------------------- z-march
// Up to two boxes per launch: work-groups [0, split_block) tile box 0, the
// rest tile box 1 (the two x slabs of the boundary go in one launch).
struct ZBox {
    Box b;
    int xa;        // first x of the tile grid (b.i0 rounded down to the vector width)
    int ntx, nty;  // tiles in x and y
};
struct ZTile {
    ZBox box[2];
    int64_t split_block;
    int nx, ny;   // array sizes in x and y
    int zc;       // planes per work-group
    int remap;    // XCD-aware renumbering of work-groups
    int rblock;   // mode 2: x-rows of tiles per block dealt to one XCD
    // wrapped x-slab tiles (WRAP): virtual row j holds the last w2 points of
    // row j-1 and the first w2 points of row j, which sit next to each other
    // in memory; points of the left part are computed where x is in
    // [wl0, wl1) and row j-1 is in [jr0, jr1), of the right part where x is
    // in [wr0, wr1) and row j is in [jr0, jr1).  With wh set the tile also
    // loads its outer x neighbours: x = -1 is column nx-w2-1 of row j-1 and
    // x = 2*w2 is column w2 of row j (slabs a full half tile wide).
    int w2, wl0, wl1, wr0, wr1, jr0, jr1, wh;
    XHalo xh;
    SrOrigin so;
    // boundary slabs in the same launch: work-groups [0, slab_blocks) run
    // the slab waves of ss (dispatched first), the rest tile the boxes
    int64_t slab_blocks;
    SlabSet ss;
};

// BX x TY threads; thread (tx, ty) owns RY consecutive rows of VEC points.
// Tile: TW = BX*VEC points by TH = TY*RY rows; the LDS plane tile adds one
// halo row above and below (loaded by thread rows 0 and TY-1) and one halo
// column left and right (loaded by lanes tx = 0 and BX-1).
template <typename S, int VEC, int BX, int TY, int RY, int WRAP, int SR>
__global__ void __launch_bounds__(BX *TY)
k_step_zmarch(S *__restrict__ T2, const S *__restrict__ T, const S *__restrict__ Ci, ZTile z,
              compute_t<S> a, compute_t<S> rx, compute_t<S> ry, compute_t<S> rz, uint32_t key)
{
    constexpr int stochastic = SR;
    using C = compute_t<S>;
    using V = typename VecOf<S, VEC>::type;
    // Interior columns of the LDS tile from P0, halo columns at P0-1 and
    // P0+TW.  Where a vector is 16 bytes of C (FP64, and FP16 widened to
    // FP32) the interior starts 16-byte aligned, so each vector is one LDS
    // access (512^3: FP64 0.5294 -> 0.5284 ms, FP16 with stochastic rounding
    // 0.1651 -> 0.1621; FP32 was no faster and keeps P0 = 1).
    constexpr int P0 = (VEC * (int)sizeof(C) == 16 && sizeof(S) != 4) ? 16 / (int)sizeof(C) : 1;
    constexpr int TW = BX * VEC, TH = TY * RY, LH = TH + 2, LW = TW + 2 * P0;
    __shared__ __attribute__((aligned(16))) C tile[2][LH][LW];

    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    int64_t g = blockIdx.x;
    if constexpr (!WRAP) {
        if (g < z.slab_blocks) {
            slab_body<S, VEC, (SR > 0)>(T2, T, Ci, z.ss, a, rx, ry, rz, key,
                                        g * (BX * TY / 64) + (int64_t)(threadIdx.x / 64), threadIdx.x & 63);
            return;
        }
    }
    g -= z.slab_blocks;
    const int64_t nblk = gridDim.x - z.slab_blocks;
    if (z.remap == 1) {
        g = xcd_remap(g, nblk);
    } else if (z.remap >= 2) {
        // keep each x-row of tiles on one XCD (work-group g runs on XCD g % 8),
        // so neighbouring tiles read each other's edge lines from the same L2;
        // mode 2 deals rows to XCDs in turn, mode 3 in contiguous ranges
        const int64_t ntx0 = z.box[0].ntx, B = z.rblock;
        const int64_t P = nblk / ntx0, P8 = z.remap == 2 ? P / (8 * B) * (8 * B) : P / 8 * 8;
        if (g < ntx0 * P8) {
            const int64_t x = g % 8, slot = g / 8;
            const int64_t q = slot / ntx0;
            const int64_t p = z.remap == 2 ? ((q / B) * 8 + x) * B + q % B : x * (P8 / 8) + q;
            g = slot % ntx0 + ntx0 * p;
        }
    }
    const int q1 = g >= z.split_block;
    if (q1) g -= z.split_block;
    const Box bb = q1 ? z.box[1].b : z.box[0].b;
    const int xa = q1 ? z.box[1].xa : z.box[0].xa;
    const int ntx = q1 ? z.box[1].ntx : z.box[0].ntx;
    const int nty = q1 ? z.box[1].nty : z.box[0].nty;
    const int bx = (int)(g % ntx);
    const int64_t rest = g / ntx;
    const int by = (int)(rest % nty);
    const int bz = (int)(rest / nty);

    const int nx = z.nx, ny = z.ny;
    const int64_t sxy = (int64_t)nx * ny;
    const int x0 = xa + bx * TW;
    const int i = x0 + tx * VEC;
    const bool xin = i < nx;
    const int jb = bb.j0 + by * TH;  // first row of the tile
    const int kb = bb.k0 + bz * z.zc;
    const int ke = (kb + z.zc < bb.k1) ? kb + z.zc : bb.k1;
    int64_t col[RY];
    int jr[RY];
    bool crow[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        jr[r] = jb + ty * RY + r;
        const int jc = jr[r] > ny - 1 ? ny - 1 : jr[r];
        col[r] = (int64_t)jc * nx + i;
        crow[r] = jr[r] < bb.j1;
    }
    // y-halo row of this thread row (thread rows 0 and TY-1 only)
    const bool hy = ty == 0 || ty == TY - 1;
    const int jh = (ty == 0) ? jb - 1 : (jb + TH > ny - 1 ? ny - 1 : jb + TH);
    const int64_t colhy = (int64_t)jh * nx + i;
    const int hyrow = (ty == 0) ? 0 : LH - 1;
    // x-halo points of this thread's rows (lanes 0 and BX-1 only); a wrapped
    // tile needs them only when a slab fills its half tile
    const bool own_h = WRAP ? (z.wh && (tx == 0 || tx == BX - 1))
                            : ((tx == 0 && x0 >= 1) || (tx == BX - 1 && x0 + TW < nx));
    const int xh = (tx == 0) ? x0 - 1 : x0 + TW;
    const int hcol = (tx == 0) ? P0 - 1 : P0 + TW;

    auto ldv = [&](const S *A, int k, int64_t c) -> V {
        V v{};
        if (xin) v = *reinterpret_cast<const V *>(A + (int64_t)k * sxy + c);
        return v;
    };
    // Ci and T2 are touched once per step: non-temporal loads and stores keep
    // them from displacing the T lines that neighbouring tiles reuse
    auto ldv_nt = [&](const S *A, int k, int64_t c) -> V {
        V v{};
        if (xin) v = __builtin_nontemporal_load(reinterpret_cast<const V *>(A + (int64_t)k * sxy + c));
        return v;
    };

    // T of planes k-1, k, k+1 per row, Ci of plane k, halo values of plane k
    V tm[RY], tc[RY], tp[RY], ci[RY];
    S hx[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        tm[r] = ldv(T, kb - 1, col[r]);
        tc[r] = ldv(T, kb, col[r]);
        tp[r] = ldv(T, kb + 1, col[r]);
        ci[r] = crow[r] ? ldv_nt(Ci, kb, col[r]) : V{};
        hx[r] = own_h ? T[(int64_t)kb * sxy + col[r] - i + xh] : S(0);
    }
    V yh = hy ? ldv(T, kb, colhy) : V{};
    // SR == 2 (rows of 4-point vectors whose global x origin and x period
    // are even, so every vector holds two whole hash pairs): the hash input
    // multiple of each row's first pair, fixed for the march, and the step
    // from a vector's first pair to its second
    uint32_t hmul[RY], hstep = 0;
    if constexpr (SR == 2) {
        static_assert(VEC == 4 && !WRAP, "whole pairs need 4-point vectors");
        const int g0 = sr_wrap(i + z.so.ox, z.so.px), g2 = sr_wrap(i + 2 + z.so.ox, z.so.px);
        hstep = (uint32_t)((g2 >> 1) - (g0 >> 1)) * kPcgMul;
#pragma unroll
        for (int r = 0; r < RY; ++r) hmul[r] = sr_pair_index(g0, sr_wrap(jr[r] + z.so.oy, z.so.py), z.so) * kPcgMul;
    }

    // SR == 2, one plane: every row computed and rounded before the stores
    // (a row past the box computes values it does not store), each vector
    // with the instruction, and all RY vectors redone in round_sr when one
    // of their values lies outside the FP16 normal range: one test and no
    // branch per value in the common case
    auto sr2_rows = [&](int k, int buf, uint32_t pk) {
      if constexpr (SR == 2) {
        typedef _Float16 H2 __attribute__((ext_vector_type(2)));
        const uint32_t pmul = pk * kPcgMul + kPcgInc;
        C v[RY][VEC];
        uint32_t w[RY][VEC];
        V out[RY];
        bool normal = true;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int lr = 1 + ty * RY + r;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int lc = P0 + tx * VEC + q;
                const C c = widen<C>(lane_elem<S, VEC>(tc[r], q));
                const C xm = (q == 0) ? tile[buf][lr][lc - 1] : widen<C>(lane_elem<S, VEC>(tc[r], q - 1));
                const C xp = (q == VEC - 1) ? tile[buf][lr][lc + 1] : widen<C>(lane_elem<S, VEC>(tc[r], q + 1));
                const C ym = (r == 0) ? tile[buf][lr - 1][lc] : widen<C>(lane_elem<S, VEC>(tc[r - 1], q));
                const C yp = (r == RY - 1) ? tile[buf][lr + 1][lc] : widen<C>(lane_elem<S, VEC>(tc[r + 1], q));
                v[r][q] = diffuse<C>(c, xm, xp, ym, yp, widen<C>(lane_elem<S, VEC>(tm[r], q)),
                                     widen<C>(lane_elem<S, VEC>(tp[r], q)), widen<C>(lane_elem<S, VEC>(ci[r], q)), a,
                                     rx, ry, rz);
            }
            const uint32_t s0 = hmul[r] + pmul;
            w[r][0] = pcg_permute(s0);
            w[r][1] = w[r][0] << 16;
            w[r][2] = pcg_permute(s0 + hstep);
            w[r][3] = w[r][2] << 16;
            H2 h0 = __builtin_bit_cast(H2, w[r][0]), h1 = __builtin_bit_cast(H2, w[r][2]);
            h0 = __builtin_amdgcn_cvt_sr_f16_f32(h0, v[r][0], w[r][0], false);
            h0 = __builtin_amdgcn_cvt_sr_f16_f32(h0, v[r][1], w[r][1], true);
            h1 = __builtin_amdgcn_cvt_sr_f16_f32(h1, v[r][2], w[r][2], false);
            h1 = __builtin_amdgcn_cvt_sr_f16_f32(h1, v[r][3], w[r][3], true);
            out[r] = __builtin_shufflevector(h0, h1, 0, 1, 2, 3);
            normal = normal && sr_normal4(v[r]);
        }
        if (!normal) {
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int q = 0; q < VEC; ++q) out[r][q] = round_sr(v[r][q], w[r][q]);
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!crow[r]) continue;
            S *dst = T2 + (int64_t)k * sxy + col[r];
            if (xin && i >= bb.i0 && i + VEC <= bb.i1) {
                __builtin_nontemporal_store(out[r], reinterpret_cast<V *>(dst));
            } else if (xin) {
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (i + q >= bb.i0 && i + q < bb.i1) dst[q] = out[r][q];
            }
            // the x exchange fused into the store, as below
            if (z.xh.on_lo && xin && i <= z.xh.lo && i + VEC > z.xh.lo) {
                const int q = z.xh.lo - i;
                if (i + q >= bb.i0 && i + q < bb.i1)
                    dst[q + nx - 1 - z.xh.lo + z.xh.d_lo] = lane_elem_dyn<S, VEC>(out[r], q);
            }
            if (z.xh.on_hi && xin && i <= z.xh.hi && i + VEC > z.xh.hi) {
                const int q = z.xh.hi - i;
                if (i + q >= bb.i0 && i + q < bb.i1) dst[q - z.xh.hi + z.xh.d_hi] = lane_elem_dyn<S, VEC>(out[r], q);
            }
        }
      }
    };

    for (int k = kb; k < ke; ++k) {
        const int buf = (k - kb) & 1;
        const bool more = k + 1 < ke;
        // loads for the next plane, consumed one iteration later
        V tn[RY], cn[RY], yn{};
        S hn[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            tn[r] = more ? ldv(T, k + 2, col[r]) : V{};
            cn[r] = (more && crow[r]) ? ldv_nt(Ci, k + 1, col[r]) : V{};
            hn[r] = (more && own_h) ? T[(int64_t)(k + 1) * sxy + col[r] - i + xh] : S(0);
        }
        if (more && hy) yn = ldv(T, k + 1, colhy);
        // plane k into LDS
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int q = 0; q < VEC; ++q)
                tile[buf][1 + ty * RY + r][P0 + tx * VEC + q] = widen<C>(lane_elem<S, VEC>(tc[r], q));
            if (own_h) tile[buf][1 + ty * RY + r][hcol] = widen<C>(hx[r]);
        }
        if (hy) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[buf][hyrow][P0 + tx * VEC + q] = widen<C>(lane_elem<S, VEC>(yh, q));
        }
        __syncthreads();
        const uint32_t pk = stochastic ? sr_plane_key(key, k, z.so) : 0u;
        if constexpr (SR == 2) {
            sr2_rows(k, buf, pk);
        } else {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!crow[r]) continue;
            const int lr = 1 + ty * RY + r;
            uint32_t rbits[VEC];
            if constexpr (SR) {
                if constexpr (!WRAP && VEC % 2 == 0) {
#pragma unroll
                    for (int q = 0; q < VEC; q += 2) sr_point_bits2(pk, i + q, jr[r], z.so, rbits[q], rbits[q + 1]);
                } else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        int ir = i + q, jreal = jr[r];
                        if (WRAP) {
                            const bool left = ir < z.w2;
                            ir = left ? ir + nx - z.w2 : ir - z.w2;
                            jreal = left ? jreal - 1 : jreal;
                        }
                        rbits[q] = sr_point_bits(pk, ir, jreal, z.so);
                    }
                }
            }
            V out;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int lc = P0 + tx * VEC + q;
                const C c = widen<C>(lane_elem<S, VEC>(tc[r], q));
                const C xm = (q == 0) ? tile[buf][lr][lc - 1] : widen<C>(lane_elem<S, VEC>(tc[r], q - 1));
                const C xp = (q == VEC - 1) ? tile[buf][lr][lc + 1] : widen<C>(lane_elem<S, VEC>(tc[r], q + 1));
                const C ym = (r == 0) ? tile[buf][lr - 1][lc] : widen<C>(lane_elem<S, VEC>(tc[r - 1], q));
                const C yp = (r == RY - 1) ? tile[buf][lr + 1][lc] : widen<C>(lane_elem<S, VEC>(tc[r + 1], q));
                const C v = diffuse<C>(c, xm, xp, ym, yp, widen<C>(lane_elem<S, VEC>(tm[r], q)),
                                       widen<C>(lane_elem<S, VEC>(tp[r], q)), widen<C>(lane_elem<S, VEC>(ci[r], q)),
                                       a, rx, ry, rz);
                set_elem<S, VEC>(out, q, Store<S>::put(v, stochastic ? rbits[q] : 0u, stochastic));
            }
            S *dst = T2 + (int64_t)k * sxy + col[r];
            // dst + q is the point's own address; ix is its x index in the row
            int ix = i;
            bool rowin = xin;
            int c0 = bb.i0, c1 = bb.i1;
            if (WRAP) {
                // VEC divides w2, so a vector lies in one part
                const bool left = i < z.w2;
                const int jreal = left ? jr[r] - 1 : jr[r];
                ix = left ? i + nx - z.w2 : i - z.w2;
                rowin = xin && jreal >= z.jr0 && jreal < z.jr1;
                c0 = left ? z.wl0 : z.wr0;
                c1 = left ? z.wl1 : z.wr1;
                if (rowin) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q)
                        if (i + q >= c0 && i + q < c1) dst[q] = lane_elem<S, VEC>(out, q);
                }
            } else if (xin && i >= bb.i0 && i + VEC <= bb.i1) {
                __builtin_nontemporal_store(out, reinterpret_cast<V *>(dst));
            } else if (xin) {
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (i + q >= bb.i0 && i + q < bb.i1) dst[q] = lane_elem<S, VEC>(out, q);
            }
            // x exchange fused into the store: the point at x = ol-1 also
            // fills x = nx-1 of the lower x neighbour, the point at x = nx-ol
            // x = 0 of the upper one (this array itself on one periodic rank)
            if (z.xh.on_lo && rowin && ix <= z.xh.lo && ix + VEC > z.xh.lo) {
                const int q = z.xh.lo - ix;
                if (i + q >= c0 && i + q < c1)
                    dst[q + nx - 1 - z.xh.lo + z.xh.d_lo] = lane_elem_dyn<S, VEC>(out, q);
            }
            if (z.xh.on_hi && rowin && ix <= z.xh.hi && ix + VEC > z.xh.hi) {
                const int q = z.xh.hi - ix;
                if (i + q >= c0 && i + q < c1) dst[q - z.xh.hi + z.xh.d_hi] = lane_elem_dyn<S, VEC>(out, q);
            }
        }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            tm[r] = tc[r];
            tc[r] = tp[r];
            tp[r] = tn[r];
            ci[r] = cn[r];
            hx[r] = hn[r];
        }
        yh = yn;
    }
}

// ------------------------------------------------------------- launchers
static int env_int(const char *name, int dflt)
{
    const char *s = getenv(name);
    return (s && *s) ? atoi(s) : dflt;
}

template <typename S>
static int run_boxes(const StepArgs &a, const Box *b, int nb, hipStream_t s)
{
    using C = compute_t<S>;
    BoxSet bs = make_boxset(b, nb);
    int64_t threads = bs.first[nb];
    if (threads == 0) return IGG_OK;
    int64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(k_step_boxes<S>, dim3((unsigned)blocks), dim3(256), 0, s, (S *)a.T2,
                       (const S *)a.T, (const S *)a.Ci, bs, a.nx, a.ny, (C)a.a, (C)a.rx, (C)a.ry,
                       (C)a.rz, a.key, a.stochastic, a.xh, a.so);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_step_boxes(int dtype, const StepArgs &a, const Box *b, int nb, hipStream_t s)
{
    if (dtype == IGG_F64) return run_boxes<double>(a, b, nb, s);
    if (dtype == IGG_F32) return run_boxes<float>(a, b, nb, s);
    return run_boxes<_Float16>(a, b, nb, s);
}

// Tile one or two boxes with TW x TH tiles and march zc planes per
// work-group.  Many short marches balance the 256 CUs, and the two extra
// planes a chunk reads are mostly served from cache: the chunk (at most 16
// planes) is halved, down to 4, while the launch would have fewer than
// min_groups work-groups.  Keeping each x-row of tiles
// on one XCD cut the inner kernel's L2 fetches by 10% and its time by 6%.
// Launch settings of one z-march launch: planes per work-group and the
// work-group to XCD mapping, each with an environment override for tuning.
struct ZLaunch {
    int zc;
    const char *zc_env;
    int remap;
    const char *remap_env;
    int64_t min_groups;
};
// FP64 inner region (and FP32 rows without vector loads): 8 planes, x-rows
// of tiles dealt to the XCDs in turn; chunks halved below 4096 work-groups
// (in a ping-pong time loop 4 planes beat 16 by 5% at 256^3 and by 6% at
// 384^3; at 512^3 8 planes beat 16 by 1% in the one-launch step and by 2%
// unsplit).
static const ZLaunch kInner = {8, "IGG_ZCHUNK", 2, "IGG_XCD_REMAP", 4096};
// FP32 inner region: 16 planes, contiguous ranges of tile rows per XCD
// (at 512^3 the 32-row tiles take 8: 2048 work-groups)
static const ZLaunch kInnerRanges = {16, "IGG_ZCHUNK", 3, "IGG_XCD_REMAP", 2048};
// FP16 inner region: the same with chunks halved below 8192 work-groups (8
// planes at 512^3: 1.5% faster than 16 in a ping-pong time loop)
static const ZLaunch kInnerF16 = {16, "IGG_ZCHUNK", 3, "IGG_XCD_REMAP", 8192};
// x slabs: 8 planes, contiguous ranges of tile rows per XCD
static const ZLaunch kXSlab = {8, "IGG_XSLAB_ZCHUNK", 3, "IGG_XSLAB_REMAP", 2048};

// The slab work of boxes b (y and z slabs) for runs of 64*VEC points, with
// the fused pack when pk is given.
// mc_fixed > 0: march chunks of that many steps (unless IGG_SLAB_MARCH is set).
template <typename S, int VEC>
static SlabSet make_slabset(const StepArgs &a, const Box *b, int nb, const SlabPack *pk, int mc_fixed = 0)
{
    constexpr int RUN = 64 * VEC;
    SlabSet ss{};
    ss.nx = a.nx;
    ss.ny = a.ny;
    ss.nz = a.nz;
    ss.xh = a.xh;
    ss.so = a.so;
    ss.n = nb;
    // each box marches along the longer of its y and z extents
    int64_t mlen[4], rows[4];
    for (int q = 0; q < nb; ++q) {
        SlabBox &sb = ss.s[q];
        sb.b = b[q];
        const int hy = b[q].j1 - b[q].j0, hz = b[q].k1 - b[q].k0;
        sb.mz = hz >= hy;
        sb.nxs = (a.nx + RUN - 1) / RUN;
        sb.nrow = sb.mz ? hy : hz;
        rows[q] = (int64_t)sb.nxs * sb.nrow;
        mlen[q] = sb.mz ? hz : hy;
    }
    auto waves = [&](int mc) {
        int64_t w = 0;
        for (int q = 0; q < nb; ++q) w += rows[q] * ((mlen[q] + mc - 1) / mc);
        return w;
    };
    int mc = env_int("IGG_SLAB_MARCH", mc_fixed);
    if (mc < 1) {
        // march chunks of 16 steps, halved (down to 2) while the launch has
        // fewer than 4096 waves
        mc = 16;
        while (mc > 2 && waves(mc) < 4096) mc /= 2;
    }
    ss.mc = mc;
    int64_t first = 0;
    for (int q = 0; q < nb; ++q) {
        ss.s[q].first = first;
        first += rows[q] * ((mlen[q] + mc - 1) / mc);
    }
    ss.waves = first;
    if (pk) {
        ss.pack = 1;
        const int64_t e = sizeof(S), nx = a.nx, ny = a.ny, nz = a.nz;
        for (int d = 0; d < 2; ++d)
            for (int side = 0; side < 2; ++side) {
                if (pk->direct) {
                    // the halo plane the sent plane fills: y side 0 -> j = ny-1,
                    // side 1 -> j = 0; z likewise
                    const int64_t plane = side == 0 ? (d == 0 ? ny - 1 : nz - 1) : 0;
                    ss.send[d][side] = (unsigned char *)a.T2 + plane * (d == 0 ? nx : nx * ny) * e;
                    ss.bstride[d] = d == 0 ? nx * ny : nx;
                } else {
                    ss.send[d][side] = pk->send[d][side];
                    ss.bstride[d] = nx;
                }
                const int dim = d + 1;
                ss.src[d][side] = side == 0 ? pk->ol[dim] - 1 : (dim == 1 ? a.ny : a.nz) - pk->ol[dim];
            }
        const int n3[3] = {a.nx, a.ny, a.nz};
        for (int d = 0; d < 3; ++d) {
            ss.img[d][0] = pk->ol[d] - 1;
            ss.img[d][1] = n3[d] - pk->ol[d];
        }
    }
    return ss;
}

template <typename S, int VEC>
static int run_slabs(const StepArgs &a, const Box *b, int nb, const SlabPack *pk, hipStream_t s)
{
    using C = compute_t<S>;
    const SlabSet ss = make_slabset<S, VEC>(a, b, nb, pk);
    if (ss.waves == 0) return IGG_OK;
    const int64_t blocks = (ss.waves + 3) / 4;
    bool sr_launched = false;
    if constexpr (std::is_same<S, _Float16>::value) {
        if (a.stochastic) {
            hipLaunchKernelGGL((k_step_slab<S, VEC, 1>), dim3((unsigned)blocks), dim3(256), 0, s, (S *)a.T2,
                               (const S *)a.T, (const S *)a.Ci, ss, (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz, a.key);
            sr_launched = true;
        }
    }
    if (!sr_launched)
        hipLaunchKernelGGL((k_step_slab<S, VEC, 0>), dim3((unsigned)blocks), dim3(256), 0, s, (S *)a.T2,
                           (const S *)a.T, (const S *)a.Ci, ss, (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz, a.key);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

template <typename S, int VEC, int BX, int TY, int RY, int WRAP = 0>
static int run_zmarch(const StepArgs &a, const Box *b, int nbox, hipStream_t s, const ZLaunch &L,
                      const ZTile *wrap = nullptr, const SlabSet *slabs = nullptr)
{
    using C = compute_t<S>;
    constexpr int TW = BX * VEC, BY = TY * RY;
    ZTile z{};
    if (wrap) z = *wrap;
    z.nx = a.nx;
    z.ny = a.ny;
    z.xh = a.xh;
    z.so = a.so;
    int64_t columns = 0;
    int depth_max = 0;
    for (int q = 0; q < nbox; ++q) {
        const int xa = (b[q].i0 / VEC) * VEC;
        columns += (int64_t)((b[q].i1 - xa + TW - 1) / TW) * ((b[q].j1 - b[q].j0 + BY - 1) / BY);
        depth_max = std::max(depth_max, b[q].k1 - b[q].k0);
    }
    int zc = env_int(L.zc_env, 0);
    if (zc < 1) zc = zchunk_for_groups(columns, depth_max, L.zc, L.min_groups);
    z.zc = zc;
    z.remap = env_int(L.remap_env, L.remap);
    z.rblock = std::max(1, env_int("IGG_XCD_BLOCK", 1));
    int64_t blocks = 0;
    z.split_block = INT64_MAX;
    for (int q = 0; q < nbox; ++q) {
        ZBox &zb = z.box[q];
        zb.b = b[q];
        zb.xa = (b[q].i0 / VEC) * VEC;
        zb.ntx = (b[q].i1 - zb.xa + TW - 1) / TW;
        zb.nty = (b[q].j1 - b[q].j0 + BY - 1) / BY;
        int depth = b[q].k1 - b[q].k0;
        int64_t nb = (int64_t)zb.ntx * zb.nty * ((depth + zc - 1) / zc);
        if (q == 1) z.split_block = blocks;
        blocks += nb;
    }
    if (nbox == 1) z.box[1] = z.box[0];
    if (slabs && slabs->waves > 0) {
        z.ss = *slabs;
        z.slab_blocks = (slabs->waves + (BX * TY / 64) - 1) / (BX * TY / 64);
        blocks += z.slab_blocks;
    }
    if (blocks == 0) return IGG_OK;
    // a wrapped tile addresses its arrays from w2 points before each row
    const int64_t off = WRAP ? z.w2 : 0;
    bool sr_launched = false;
    if constexpr (std::is_same<S, _Float16>::value && VEC == 4 && !WRAP) {
        // every 4-point vector holds two whole hash pairs when the global x
        // origin and the x period are even (vectors start at multiples of 4)
        if (a.stochastic && a.so.ox % 2 == 0 && a.so.px % 2 == 0) {
            hipLaunchKernelGGL((k_step_zmarch<S, VEC, BX, TY, RY, WRAP, 2>), dim3((unsigned)blocks), dim3(BX * TY),
                               0, s, (S *)a.T2, (const S *)a.T, (const S *)a.Ci, z, (C)a.a, (C)a.rx, (C)a.ry,
                               (C)a.rz, a.key);
            sr_launched = true;
        }
    }
    if constexpr (std::is_same<S, _Float16>::value) {
        if (a.stochastic && !sr_launched) {
            hipLaunchKernelGGL((k_step_zmarch<S, VEC, BX, TY, RY, WRAP, 1>), dim3((unsigned)blocks), dim3(BX * TY),
                               0, s, (S *)a.T2 - off, (const S *)a.T - off, (const S *)a.Ci - off, z, (C)a.a,
                               (C)a.rx, (C)a.ry, (C)a.rz, a.key);
            sr_launched = true;
        }
    }
    if (!sr_launched)
        hipLaunchKernelGGL((k_step_zmarch<S, VEC, BX, TY, RY, WRAP, 0>), dim3((unsigned)blocks), dim3(BX * TY), 0,
                           s, (S *)a.T2 - off, (const S *)a.T - off, (const S *)a.Ci - off, z, (C)a.a, (C)a.rx,
                           (C)a.ry, (C)a.rz, a.key);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

static bool aligned(const void *p, int bytes) { return ((uintptr_t)p % (uintptr_t)bytes) == 0; }

template <typename S, int VEC>
static bool vec_ok(const StepArgs &a)
{
    const int vb = (int)sizeof(S) * VEC;
    return a.nx % VEC == 0 && aligned(a.T, vb) && aligned(a.T2, vb) && aligned(a.Ci, vb);
}

// Inner region.  FP64: 128-point (1 KB) tile rows, 16-byte loads, four
// rows per thread, 32 rows per tile (512 threads; two rows per thread, 16
// rows, below 2^26 points).  FP32: 256-point (1 KB) rows, 16-byte loads, two rows per
// thread, 32 rows over 1024 threads from 2^26 points (16 rows below).
// FP16: 256-point (512-byte) rows, 8-byte loads, two rows per thread, 8
// rows (256 threads: 1-3% faster than 512-thread tiles of 16 rows at 256^3
// and 512^3; 16-byte loads over 512-point rows, or four rows per thread,
// 6-19% slower at 512^3: more registers, fewer waves).
// These shapes and work-group mappings measured fastest on MI355X at 512^3.
// Rows whose length does not allow vector loads take one point per lane;
// regions below zmarch_min_points() take the box kernel.
// One inner-region launch, with the slab waves of yz (nyz boxes) run by
// the launch's first work-groups when nyz > 0.
template <typename S, int VEC, int BX, int TY, int RY>
static int run_inner(const StepArgs &a, const Box &b, hipStream_t s, const ZLaunch &L, const Box *yz, int nyz,
                     const SlabPack *pk)
{
    if (nyz == 0) return run_zmarch<S, VEC, BX, TY, RY>(a, &b, 1, s, L);
    // march chunks measured fastest for the launch at 512^3 (the slab waves
    // share it with the inner tiles, so their count matters less than the
    // rows each reloads per chunk): FP64 8 steps (0.5412 ms per step against
    // 0.5459 with 2), FP32 2 (0.2930 against 0.3036 with 8), FP16 4; FP64
    // regions below 2^26 points take 2 (256^3: 72.8 us per step against 76.1)
    const int mc = sizeof(S) == 8 ? (box_count(b) >= ((int64_t)1 << 26) ? 8 : 2) : sizeof(S) == 4 ? 2 : 4;
    const SlabSet ss = make_slabset<S, VEC>(a, yz, nyz, pk, mc);
    return run_zmarch<S, VEC, BX, TY, RY>(a, &b, 1, s, L, nullptr, &ss);
}

int launch_step_inner(int dtype, const StepArgs &a, const Box &b, hipStream_t s, const Split *slabs,
                      const SlabPack *pk)
{
    Box yz[6];
    int nyz = 0;
    if (slabs)
        for (int q = 0; q < slabs->nb; ++q)
            if (slabs->kind[q] == 1) yz[nyz++] = slabs->boundary[q];
    if (nyz > 4) return fail(IGG_ERR_ARG, "internal: more than four y/z slabs");
    if (box_count(b) < zmarch_min_points()) {
        // small grids: the slabs first, then the box kernel
        int rc;
        if (nyz && (rc = launch_step_slabs(dtype, a, *slabs, pk, s))) return rc;
        return box_count(b) > 0 ? launch_step_boxes(dtype, a, &b, 1, s) : IGG_OK;
    }
    if (dtype == IGG_F64) {
        if (vec_ok<double, 2>(a)) {
            // a 128 x 16 tile over 512 threads of 2 rows (108 registers, 4
            // waves per SIMD): 2-3% faster at 256^3 and 384^3 than 4 rows per
            // thread, 5% slower at 512^3, so regions below 2^26 points take it
            static const char *kMidEnv = "IGG_FP64_MIDTILE_MAX_POINTS";
            const char *e = getenv(kMidEnv);
            const int64_t mid_max = (e && *e) ? atoll(e) : ((int64_t)1 << 26);
            if (box_count(b) < mid_max) return run_inner<double, 2, 64, 8, 2>(a, b, s, kInner, yz, nyz, pk);
            // 32-row tiles over 512 threads of 4 rows: fewer y-halo rows per
            // point than 16-row tiles of 256 threads (512^3: 0.8% faster)
            return run_inner<double, 2, 64, 8, 4>(a, b, s, kInner, yz, nyz, pk);
        }
        return run_inner<double, 1, 64, 8, 2>(a, b, s, kInner, yz, nyz, pk);
    }
    if (dtype == IGG_F32) {
        if (vec_ok<float, 4>(a)) {
            // 256 x 32 tiles over 1024 threads of 2 rows for regions of at
            // least 2^26 points (4% faster than 256 x 16 tiles at 512^3)
            if (box_count(b) >= ((int64_t)1 << 26))
                return run_inner<float, 4, 64, 16, 2>(a, b, s, kInnerRanges, yz, nyz, pk);
            return run_inner<float, 4, 64, 8, 2>(a, b, s, kInnerRanges, yz, nyz, pk);
        }
        return run_inner<float, 1, 64, 8, 2>(a, b, s, kInner, yz, nyz, pk);
    }
    if (vec_ok<_Float16, 4>(a)) return run_inner<_Float16, 4, 64, 4, 2>(a, b, s, kInnerF16, yz, nyz, pk);
    return run_inner<_Float16, 1, 64, 8, 2>(a, b, s, kInnerF16, yz, nyz, pk);
}

// x slabs (computed first only when the x exchange is a separate pass of
// the halo update).  The end of row j-1 and the start of row j sit next to
// each other in memory, so the two x slabs of neighbouring rows form one
// wrapped
// tile of 2*W2 points (W2 = 32 or 64): one contiguous run per row pair and
// plane holding every x neighbour, instead of two narrow pieces plus two
// separate halo lines.  Wider slabs or short rows take narrow 16-point
// tiles.  The other slabs are whole rows or planes (box kernel).
template <typename S, int VEC, int W2>
static int run_xslabs_wrapped(const StepArgs &a, const Box &lo, const Box &hi, hipStream_t s)
{
    ZTile z{};
    z.w2 = W2;
    z.wl0 = hi.i0 - a.nx + W2;
    z.wl1 = hi.i1 - a.nx + W2;
    z.wr0 = lo.i0 + W2;
    z.wr1 = lo.i1 + W2;
    z.jr0 = lo.j0;
    z.jr1 = lo.j1;
    z.wh = (z.wl0 == 0 || z.wr1 == 2 * W2) ? 1 : 0;
    Box vb{0, 2 * W2, lo.j0, lo.j1 + 1, lo.k0, lo.k1};
    return run_zmarch<S, VEC, (2 * W2) / VEC, (W2 == 64 ? 8 : 16), 2, 1>(a, &vb, 1, s, kXSlab, &z);
}

static int launch_xslabs(int dtype, const StepArgs &a, const Box *b, int nb, hipStream_t s)
{
    // wrapped form: one slab on each side, same rows and planes; the slabs
    // end at most w2 points from the row's ends (w = the larger distance)
    if (nb == 2 && b[0].i0 == 1 && b[1].i1 == a.nx - 1 && b[0].j0 == b[1].j0 && b[0].j1 == b[1].j1 &&
        b[0].k0 == b[1].k0 && b[0].k1 == b[1].k1 && b[0].j0 >= 2 && b[0].j1 <= a.ny - 2) {
        const int w = std::max(b[0].i1, a.nx - b[1].i0);
        if (w <= 31 && a.nx >= 64) {
            if (dtype == IGG_F64 && vec_ok<double, 2>(a)) return run_xslabs_wrapped<double, 2, 32>(a, b[0], b[1], s);
            if (dtype == IGG_F32 && vec_ok<float, 2>(a)) return run_xslabs_wrapped<float, 2, 32>(a, b[0], b[1], s);
            if (dtype == IGG_F16 && vec_ok<_Float16, 2>(a)) return run_xslabs_wrapped<_Float16, 2, 32>(a, b[0], b[1], s);
        }
        if (w <= 64 && a.nx >= 130) {
            if (dtype == IGG_F64 && vec_ok<double, 2>(a)) return run_xslabs_wrapped<double, 2, 64>(a, b[0], b[1], s);
            if (dtype == IGG_F32 && vec_ok<float, 2>(a)) return run_xslabs_wrapped<float, 2, 64>(a, b[0], b[1], s);
            if (dtype == IGG_F16 && vec_ok<_Float16, 2>(a)) return run_xslabs_wrapped<_Float16, 2, 64>(a, b[0], b[1], s);
        }
    }
    if (dtype == IGG_F64) {
        if (vec_ok<double, 2>(a)) return run_zmarch<double, 2, 8, 32, 1>(a, b, nb, s, kXSlab);
        return run_zmarch<double, 1, 16, 16, 1>(a, b, nb, s, kXSlab);
    }
    if (dtype == IGG_F32) {
        if (vec_ok<float, 2>(a)) return run_zmarch<float, 2, 8, 32, 1>(a, b, nb, s, kXSlab);
        return run_zmarch<float, 1, 16, 16, 1>(a, b, nb, s, kXSlab);
    }
    if (vec_ok<_Float16, 2>(a)) return run_zmarch<_Float16, 2, 8, 32, 1>(a, b, nb, s, kXSlab);
    return run_zmarch<_Float16, 1, 16, 16, 1>(a, b, nb, s, kXSlab);
}

int launch_step_boundary(int dtype, const StepArgs &a, const Split &sp, hipStream_t s)
{
    Box xs[2], other[6];
    int nxs = 0, nother = 0;
    for (int q = 0; q < sp.nb; ++q) {
        if (sp.kind[q] == 0)
            xs[nxs++] = sp.boundary[q];
        else
            other[nother++] = sp.boundary[q];
    }
    int rc;
    if (nother && (rc = launch_step_slabs(dtype, a, sp, nullptr, s))) return rc;
    if (nxs && (rc = launch_xslabs(dtype, a, xs, nxs, s))) return rc;
    return IGG_OK;
}


int launch_step_slabs(int dtype, const StepArgs &a, const Split &sp, const SlabPack *pk, hipStream_t s)
{
    Box yz[6];
    int n = 0;
    for (int q = 0; q < sp.nb; ++q)
        if (sp.kind[q] == 1) yz[n++] = sp.boundary[q];
    if (n == 0) return IGG_OK;
    if (n > 4) return fail(IGG_ERR_ARG, "internal: more than four y/z slabs");
    if (dtype == IGG_F64) {
        if (vec_ok<double, 2>(a)) return run_slabs<double, 2>(a, yz, n, pk, s);
        return run_slabs<double, 1>(a, yz, n, pk, s);
    }
    if (dtype == IGG_F32) {
        if (vec_ok<float, 4>(a)) return run_slabs<float, 4>(a, yz, n, pk, s);
        return run_slabs<float, 1>(a, yz, n, pk, s);
    }
    if (vec_ok<_Float16, 8>(a)) return run_slabs<_Float16, 8>(a, yz, n, pk, s);
    return run_slabs<_Float16, 1>(a, yz, n, pk, s);
}

}  // namespace igg
