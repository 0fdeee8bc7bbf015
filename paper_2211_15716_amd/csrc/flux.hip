// flux.hip -- staggered-grid flux form of the diffusion step (Sec. 2 on the
// regular staggered grid): face fluxes q = -lam*grad(T) and the cell update
// T2 = T - dt*Ci*div(q), in one pass per cell.  Its adjoint runs in
// adjoint.hip (the same kernels as the Laplacian form's adjoint).
//
// Sizes: cells (nx,ny,nz); qx (nx+1,ny,nz), qy (nx,ny+1,nz), qz (nx,ny,nz+1).
// Face f of a dimension lies between cells f-1 and f; fluxes are computed on
// faces 1..n-1 of the inner rows of the other two dimensions.
#include <stdlib.h>

#include "host.hpp"

namespace igg {

// Cell grid size (the face fields add one point in their own dimension).
struct FaceGeom {
    int nx, ny, nz;
};

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// ------------------------------------------------------------ fused step
// One pass per cell (i, j, k): its lower faces qx[i], qy[j], qz[k] (and the
// upper face where the cell is the last of its row, column or plane), the
// update T2 = T - dt*Ci*div(q) from the cell's six faces, and the x
// exchange of all four fields with the x neighbours (FluxXH).  The faces
// come from one expression (face_flux) and the divergence sums in a fixed
// order (flux_div), so every value equals a face pass followed by a cell
// pass.

// Stores of one cell that are not plain per-cell stores: the upper faces at
// the ends and the x-exchange copies.  p: the cell's offset in a cell-sized
// array, px and py: its lower faces' offsets in qx and qy.
template <typename C>
__device__ __forceinline__ void flux_extra_stores(C *T2, C *qx, C *qy, C *qz, int i, int j, int k,
                                                  int64_t p, int64_t px, int64_t py, const FaceGeom &g,
                                                  const FluxXH &xh, C v2, C qxl, C qxu, C qyl, C qyu,
                                                  C qzl, C qzu)
{
    const int nx = g.nx;
    const int64_t sz = (int64_t)nx * g.ny;
    const bool lastx = i == nx - 2, lasty = j == g.ny - 2, lastz = k == g.nz - 2;
    if (lastx) qx[px + 1] = qxu;
    if (lasty) qy[py + nx] = qyu;
    if (lastz) qz[p + sz] = qzu;
    // T2, qy, qz: column ol-1 -> lower neighbour's nx-1, column nx-ol ->
    // upper neighbour's 0
    for (int side = 0; side < 2; ++side) {
        if (!(side == 0 ? xh.on_lo : xh.on_hi)) continue;
        const int src = side == 0 ? xh.ol - 1 : nx - xh.ol;
        if (i != src) continue;
        const int64_t sh = side == 0 ? (int64_t)(nx - 1 - i) : -(int64_t)i;
        const int64_t *d = side == 0 ? xh.d_lo : xh.d_hi;
        T2[p + sh + d[0]] = v2;
        qy[py + sh + d[2]] = qyl;
        qz[p + sh + d[3]] = qzl;
        if (lasty) qy[py + nx + sh + d[2]] = qyu;
        if (lastz) qz[p + sz + sh + d[3]] = qzu;
    }
    // qx: face ol -> lower neighbour's nx, face nx-ol -> upper neighbour's 0
    // (faces i, and i+1 at the last cell)
    for (int f = i; f <= (lastx ? i + 1 : i); ++f) {
        const C v = f == i ? qxl : qxu;
        const int64_t pf = px + (f - i);
        if (xh.on_lo && f == xh.ol) qx[pf + (nx - f) + xh.d_lo[1]] = v;
        if (xh.on_hi && f == nx - xh.ol) qx[pf - f + xh.d_hi[1]] = v;
    }
}

template <typename C>
__global__ void __launch_bounds__(256)
k_flux_fused_boxes(C *__restrict__ T2, C *__restrict__ qx, C *__restrict__ qy, C *__restrict__ qz,
                   const C *__restrict__ T, const C *__restrict__ Ci, BoxSet bs, FaceGeom g, FluxXH xh, C lam,
                   C dt, C rdx, C rdy, C rdz)
{
    int i, j, k;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!boxset_point(bs, t, i, j, k)) return;
    const int nx = g.nx, ny = g.ny;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t p = i + sy * j + sz * k;
    const C t0 = T[p];
    const C qxl = face_flux<C>(t0, T[p - 1], lam, rdx), qxu = face_flux<C>(T[p + 1], t0, lam, rdx);
    const C qyl = face_flux<C>(t0, T[p - sy], lam, rdy), qyu = face_flux<C>(T[p + sy], t0, lam, rdy);
    const C qzl = face_flux<C>(t0, T[p - sz], lam, rdz), qzu = face_flux<C>(T[p + sz], t0, lam, rdz);
    const C v2 = fma_(-dt * Ci[p], flux_div<C>(qxl, qxu, qyl, qyu, qzl, qzu, rdx, rdy, rdz), t0);
    const int64_t px = i + (int64_t)(nx + 1) * (j + (int64_t)ny * k);
    const int64_t py = i + (int64_t)nx * (j + (int64_t)(ny + 1) * k);
    T2[p] = v2;
    qx[px] = qxl;
    qy[py] = qyl;
    qz[p] = qzl;
    flux_extra_stores<C>(T2, qx, qy, qz, i, j, k, p, px, py, g, xh, v2, qxl, qxu, qyl, qyu, qzl, qzu);
}

template <typename C, int VEC> struct FVec {
    typedef C type __attribute__((ext_vector_type(VEC)));
};
template <typename C> struct FVec<C, 1> {
    typedef C type;
};
template <typename C, int VEC>
__device__ __forceinline__ C fel(const typename FVec<C, VEC>::type &v, int q)
{
    if constexpr (VEC == 1)
        return v;
    else
        return v[q];
}
template <typename C, int VEC>
__device__ __forceinline__ void fset(typename FVec<C, VEC>::type &v, int q, C x)
{
    if constexpr (VEC == 1)
        v = x;
    else
        v[q] = x;
}

struct FluxTile {
    Box b;
    int xa, ntx, nty, zc, remap;
    FaceGeom g;
    FluxXH xh;
};

// z-march of the fused step: BX x TY threads, RY rows of VEC cells each;
// T of planes k-1, k, k+1 (k+2 in flight) in registers, plane k in a
// double-buffered LDS tile for the x and y neighbours (the forward step
// kernel's scheme).  T2, qy, qz leave as vectors where the cells of a
// vector all lie in the box; qx rows are nx+1 long, so its stores are per
// cell.
template <typename C, int VEC, int BX, int TY, int RY>
__global__ void __launch_bounds__(BX *TY)
k_flux_fused_zmarch(C *__restrict__ T2, C *__restrict__ qx, C *__restrict__ qy, C *__restrict__ qz,
                    const C *__restrict__ T, const C *__restrict__ Ci, FluxTile z, C lam, C dt, C rdx, C rdy,
                    C rdz)
{
    using V = typename FVec<C, VEC>::type;
    constexpr int TW = BX * VEC, TH = TY * RY, LH = TH + 2, LW = TW + 2;
    __shared__ C tile[2][LH][LW];
    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    int64_t gidx = blockIdx.x;
    if (z.remap == 2) {  // x-rows of tiles dealt to the XCDs in turn
        const int64_t ntx0 = z.ntx, P = gridDim.x / ntx0, P8 = P / 8 * 8;
        if (gidx < ntx0 * P8) {
            const int64_t x = gidx % 8, slot = gidx / 8;
            gidx = slot % ntx0 + ntx0 * (x + 8 * (slot / ntx0));
        }
    }
    const int bx = (int)(gidx % z.ntx);
    const int64_t rest = gidx / z.ntx;
    const int by = (int)(rest % z.nty);
    const int bz = (int)(rest / z.nty);
    const int nx = z.g.nx, ny = z.g.ny;
    const int64_t sxy = (int64_t)nx * ny;
    const int x0 = z.xa + bx * TW;
    const int i = x0 + tx * VEC;
    const bool xin = i < nx;
    const int jb = z.b.j0 + by * TH;
    const int kb = z.b.k0 + bz * z.zc;
    const int ke = (kb + z.zc < z.b.k1) ? kb + z.zc : z.b.k1;
    int64_t col[RY];
    int jr[RY];
    bool crow[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        jr[r] = jb + ty * RY + r;
        col[r] = (int64_t)(jr[r] > ny - 1 ? ny - 1 : jr[r]) * nx + i;
        crow[r] = jr[r] < z.b.j1;
    }
    const bool hy = ty == 0 || ty == TY - 1;
    const int jh = (ty == 0) ? jb - 1 : (jb + TH > ny - 1 ? ny - 1 : jb + TH);
    const int64_t colhy = (int64_t)jh * nx + i;
    const int hyrow = (ty == 0) ? 0 : LH - 1;
    const bool own_h = (tx == 0 && x0 >= 1) || (tx == BX - 1 && x0 + TW < nx);
    const int xh = (tx == 0) ? x0 - 1 : x0 + TW;
    const int hcol = (tx == 0) ? 0 : LW - 1;

    auto ld = [&](const C *A, int k, int64_t c) -> V {
        V v{};
        if (xin) v = *reinterpret_cast<const V *>(A + (int64_t)k * sxy + c);
        return v;
    };
    auto ld_nt = [&](const C *A, int k, int64_t c) -> V {
        V v{};
        if (xin) v = __builtin_nontemporal_load(reinterpret_cast<const V *>(A + (int64_t)k * sxy + c));
        return v;
    };

    V tm[RY], tc[RY], tp[RY], ci[RY];
    C hx[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        tm[r] = ld(T, kb - 1, col[r]);
        tc[r] = ld(T, kb, col[r]);
        tp[r] = ld(T, kb + 1, col[r]);
        ci[r] = crow[r] ? ld_nt(Ci, kb, col[r]) : V{};
        hx[r] = own_h ? T[(int64_t)kb * sxy + col[r] - i + xh] : C(0);
    }
    V yh = hy ? ld(T, kb, colhy) : V{};

    for (int k = kb; k < ke; ++k) {
        const int buf = (k - kb) & 1;
        const bool more = k + 1 < ke;
        V tn[RY], cn[RY], yn{};
        C hn[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            tn[r] = more ? ld(T, k + 2, col[r]) : V{};
            cn[r] = (more && crow[r]) ? ld_nt(Ci, k + 1, col[r]) : V{};
            hn[r] = (more && own_h) ? T[(int64_t)(k + 1) * sxy + col[r] - i + xh] : C(0);
        }
        if (more && hy) yn = ld(T, k + 1, colhy);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[buf][1 + ty * RY + r][1 + tx * VEC + q] = fel<C, VEC>(tc[r], q);
            if (own_h) tile[buf][1 + ty * RY + r][hcol] = hx[r];
        }
        if (hy) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[buf][hyrow][1 + tx * VEC + q] = fel<C, VEC>(yh, q);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!crow[r] || !xin) continue;
            const int lr = 1 + ty * RY + r;
            V o2, oy, oz;
            C oxl[VEC], oxu[VEC], oyu[VEC], ozu[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int lc = 1 + tx * VEC + q;
                const C t0 = fel<C, VEC>(tc[r], q);
                const C txm = (q == 0) ? tile[buf][lr][lc - 1] : fel<C, VEC>(tc[r], q - 1);
                const C txp = (q == VEC - 1) ? tile[buf][lr][lc + 1] : fel<C, VEC>(tc[r], q + 1);
                const C tym = (r == 0) ? tile[buf][lr - 1][lc] : fel<C, VEC>(tc[r - 1], q);
                const C typ = (r == RY - 1) ? tile[buf][lr + 1][lc] : fel<C, VEC>(tc[r + 1], q);
                const C qxl = face_flux<C>(t0, txm, lam, rdx), qxu = face_flux<C>(txp, t0, lam, rdx);
                const C qyl = face_flux<C>(t0, tym, lam, rdy), qyu = face_flux<C>(typ, t0, lam, rdy);
                const C qzl = face_flux<C>(t0, fel<C, VEC>(tm[r], q), lam, rdz);
                const C qzu = face_flux<C>(fel<C, VEC>(tp[r], q), t0, lam, rdz);
                const C v2 =
                    fma_(-dt * fel<C, VEC>(ci[r], q), flux_div<C>(qxl, qxu, qyl, qyu, qzl, qzu, rdx, rdy, rdz), t0);
                fset<C, VEC>(o2, q, v2);
                fset<C, VEC>(oy, q, qyl);
                fset<C, VEC>(oz, q, qzl);
                oxl[q] = qxl;
                oxu[q] = qxu;
                oyu[q] = qyu;
                ozu[q] = qzu;
            }
            const int j = jr[r];
            const int64_t p = (int64_t)k * sxy + col[r];
            const int64_t px = i + (int64_t)(nx + 1) * (j + (int64_t)ny * k);
            const int64_t py = i + (int64_t)nx * (j + (int64_t)(ny + 1) * k);
            const bool full = i >= z.b.i0 && i + VEC <= z.b.i1;
            if (full) {
                __builtin_nontemporal_store(o2, reinterpret_cast<V *>(T2 + p));
                __builtin_nontemporal_store(oy, reinterpret_cast<V *>(qy + py));
                __builtin_nontemporal_store(oz, reinterpret_cast<V *>(qz + p));
            }
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int ii = i + q;
                if (ii < z.b.i0 || ii >= z.b.i1) continue;
                if (!full) {
                    T2[p + q] = fel<C, VEC>(o2, q);
                    qy[py + q] = fel<C, VEC>(oy, q);
                    qz[p + q] = fel<C, VEC>(oz, q);
                }
                qx[px + q] = oxl[q];
                if (ii == nx - 2 || j == ny - 2 || k == z.g.nz - 2 ||
                    ((z.xh.on_lo || z.xh.on_hi) && (ii <= z.xh.ol || ii >= nx - z.xh.ol)))
                    flux_extra_stores<C>(T2, qx, qy, qz, ii, j, k, p + q, px + q, py + q, z.g, z.xh,
                                         fel<C, VEC>(o2, q), oxl[q], oxu[q], fel<C, VEC>(oy, q), oyu[q],
                                         fel<C, VEC>(oz, q), ozu[q]);
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

static int env_int_flux(const char *name, int dflt)
{
    const char *s = getenv(name);
    return (s && *s) ? atoi(s) : dflt;
}

template <typename C>
static int run_fused_boxes(const FluxArgs &a, const Box *b, int nb, hipStream_t s)
{
    BoxSet bs = make_boxset(b, nb);
    const int64_t threads = bs.first[nb];
    if (threads == 0) return IGG_OK;
    FaceGeom g{a.nx, a.ny, a.nz};
    hipLaunchKernelGGL(k_flux_fused_boxes<C>, dim3(blocks_for(threads)), dim3(256), 0, s, (C *)a.T2, (C *)a.qx,
                       (C *)a.qy, (C *)a.qz, (const C *)a.T, (const C *)a.Ci, bs, g, a.xh, (C)a.lam, (C)a.dt,
                       (C)a.rdx, (C)a.rdy, (C)a.rdz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

template <typename C, int VEC, int BX, int TY, int RY>
static int run_fused_zmarch(const FluxArgs &a, const Box &b, hipStream_t s)
{
    constexpr int TW = BX * VEC, TH = TY * RY;
    FluxTile z{};
    z.b = b;
    z.g = FaceGeom{a.nx, a.ny, a.nz};
    z.xh = a.xh;
    z.xa = (b.i0 / VEC) * VEC;
    z.ntx = (b.i1 - z.xa + TW - 1) / TW;
    z.nty = (b.j1 - b.j0 + TH - 1) / TH;
    const int depth = b.k1 - b.k0;
    int zc = env_int_flux("IGG_FLUX_ZCHUNK", 0);
    // chunks of 4 planes: at 768^3 (FP32) 9% faster than 16 and 4% faster
    // than 8 (the two extra planes a chunk reads mostly hit in L2)
    if (zc < 1) zc = zchunk_for_groups((int64_t)z.ntx * z.nty, depth, 4);
    z.zc = zc;
    z.remap = env_int_flux("IGG_FLUX_REMAP", 2);
    const int64_t blocks = (int64_t)z.ntx * z.nty * ((depth + zc - 1) / zc);
    if (blocks <= 0) return IGG_OK;
    hipLaunchKernelGGL((k_flux_fused_zmarch<C, VEC, BX, TY, RY>), dim3((unsigned)blocks), dim3(BX * TY), 0, s,
                       (C *)a.T2, (C *)a.qx, (C *)a.qy, (C *)a.qz, (const C *)a.T, (const C *)a.Ci, z, (C)a.lam,
                       (C)a.dt, (C)a.rdx, (C)a.rdy, (C)a.rdz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

// 16-byte vectors of `vec` cells: rows a whole number of vectors long and
// every cell-sized array (and qy, qz) 16-byte aligned
static bool flux_vec_ok(const FluxArgs &a, int vec)
{
    auto al = [](const void *p) { return ((uintptr_t)p % 16) == 0; };
    return a.nx % vec == 0 && al(a.T) && al(a.T2) && al(a.Ci) && al(a.qy) && al(a.qz);
}

int launch_flux_boxes(int dtype, const FluxArgs &a, const Box *b, int nb, hipStream_t s)
{
    return dtype == IGG_F64 ? run_fused_boxes<double>(a, b, nb, s) : run_fused_boxes<float>(a, b, nb, s);
}

// The inner region: z-march tiles of 1 KB rows (128 FP64 or 256 FP32 cells)
// where rows allow 16-byte vectors, else one cell per lane; regions below
// zmarch_min_points() take the box kernel.
int launch_flux_inner(int dtype, const FluxArgs &a, const Box &b, hipStream_t s)
{
    if (box_count(b) < zmarch_min_points()) return launch_flux_boxes(dtype, a, &b, 1, s);
    if (dtype == IGG_F64)
        return flux_vec_ok(a, 2) ? run_fused_zmarch<double, 2, 64, 4, 2>(a, b, s)
                                  : run_fused_zmarch<double, 1, 64, 4, 2>(a, b, s);
    return flux_vec_ok(a, 4) ? run_fused_zmarch<float, 4, 64, 4, 2>(a, b, s)
                              : run_fused_zmarch<float, 1, 64, 4, 2>(a, b, s);
}

}  // namespace igg
