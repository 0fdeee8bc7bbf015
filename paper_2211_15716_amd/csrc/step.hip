// step.hip -- the explicit diffusion step of Fig. 1 (`step!`) for FP64, FP32
// and FP16 storage.
//
// Two kernels compute points, both through igg::diffuse, so a point's bits
// do not depend on which of them computed it:
//   k_step_boxes   one thread per point over up to six boxes (the boundary
//                  slabs of the boundary-first schedule); plain global loads.
//   k_step_zmarch  the inner region: each work-group owns a TW x BY tile of
//                  (x, y) columns and marches up a chunk of z planes.  Every
//                  thread keeps its column's T at k-1, k, k+1 (and k+2 in
//                  flight) in registers, writes plane k to a double-buffered
//                  LDS tile, and reads its x and y neighbours from there.
//                  The tile's first and last thread rows only load the
//                  y-halo rows; two lanes per row load the x-halo points.
//                  Loads are 16 bytes per lane where the row length allows.
#include <stdlib.h>

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
             int stochastic)
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
    if (stochastic) r = point_bits(plane_key(key, k), i, j, nx);
    T2[p] = Store<S>::put(out, r, stochastic);
}

// --------------------------------------------------------------- z-march
struct ZTile {
    Box b;        // region to compute
    int nx, ny;   // array sizes in x and y
    int xa;       // first x of the tile grid (b.i0 rounded down to the vector width)
    int ntx, nty; // tiles in x and y
    int zc;       // planes per work-group
    int remap;    // XCD-aware renumbering of work-groups
};

template <typename S, int VEC, int BX, int BYT>
__global__ void __launch_bounds__(BX *BYT)
k_step_zmarch(S *__restrict__ T2, const S *__restrict__ T, const S *__restrict__ Ci, ZTile z,
              compute_t<S> a, compute_t<S> rx, compute_t<S> ry, compute_t<S> rz, uint32_t key,
              int stochastic)
{
    using C = compute_t<S>;
    using V = typename VecOf<S, VEC>::type;
    constexpr int TW = BX * VEC;  // tile width in points
    constexpr int BY = BYT - 2;   // rows computed per tile
    constexpr int LW = TW + 2;
    __shared__ C tile[2][BYT][LW];

    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    const int64_t g = z.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int bx = (int)(g % z.ntx);
    const int64_t rest = g / z.ntx;
    const int by = (int)(rest % z.nty);
    const int bz = (int)(rest / z.nty);

    const int nx = z.nx, ny = z.ny;
    const int64_t sxy = (int64_t)nx * ny;
    const int x0 = z.xa + bx * TW;
    const int i = x0 + tx * VEC;
    const int j = z.b.j0 + by * BY + ty - 1;
    const int jc = j < 0 ? 0 : (j > ny - 1 ? ny - 1 : j);
    const bool xin = i < nx;
    const bool crow = ty >= 1 && ty <= BY && j < z.b.j1;
    const int kb = z.b.k0 + bz * z.zc;
    const int ke = (kb + z.zc < z.b.k1) ? kb + z.zc : z.b.k1;
    const int64_t col = (int64_t)jc * nx + i;
    const bool hl = tx == 0 && x0 >= 1;
    const bool hr = tx == BX - 1 && x0 + TW < nx;
    const int64_t colh = (int64_t)jc * nx + (tx == 0 ? x0 - 1 : x0 + TW);
    const bool own_h = hl || hr;
    // store mask of this thread's points
    const bool full = crow && i >= z.b.i0 && i + VEC <= z.b.i1;

    auto ldv = [&](const S *A, int k) -> V {
        V v{};
        if (xin) v = *reinterpret_cast<const V *>(A + (int64_t)k * sxy + col);
        return v;
    };

    V zm = ldv(T, kb - 1), zc = ldv(T, kb), zp = ldv(T, kb + 1);
    V ci = crow ? ldv(Ci, kb) : V{};
    S h = own_h ? T[(int64_t)kb * sxy + colh] : S(0);

    for (int k = kb; k < ke; ++k) {
        const int buf = (k - kb) & 1;
        const bool more = k + 1 < ke;
        // loads for the next plane, consumed one iteration later
        V zn{}, cin{};
        S hn = S(0);
        if (more) {
            zn = ldv(T, k + 2);
            if (crow) cin = ldv(Ci, k + 1);
            if (own_h) hn = T[(int64_t)(k + 1) * sxy + colh];
        }
        // plane k into LDS
#pragma unroll
        for (int q = 0; q < VEC; ++q) tile[buf][ty][1 + tx * VEC + q] = widen<C>(lane_elem<S, VEC>(zc, q));
        if (own_h) tile[buf][ty][tx == 0 ? 0 : LW - 1] = widen<C>(h);
        __syncthreads();
        if (crow) {
            V out;
            uint32_t pk = stochastic ? plane_key(key, k) : 0u;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int lc = 1 + tx * VEC + q;
                C c = widen<C>(lane_elem<S, VEC>(zc, q));
                C xm = (q == 0) ? tile[buf][ty][lc - 1] : widen<C>(lane_elem<S, VEC>(zc, q - 1));
                C xp = (q == VEC - 1) ? tile[buf][ty][lc + 1] : widen<C>(lane_elem<S, VEC>(zc, q + 1));
                C v = diffuse<C>(c, xm, xp, tile[buf][ty - 1][lc], tile[buf][ty + 1][lc],
                                 widen<C>(lane_elem<S, VEC>(zm, q)), widen<C>(lane_elem<S, VEC>(zp, q)),
                                 widen<C>(lane_elem<S, VEC>(ci, q)), a, rx, ry, rz);
                uint32_t r = stochastic ? point_bits(pk, i + q, j, nx) : 0u;
                set_elem<S, VEC>(out, q, Store<S>::put(v, r, stochastic));
            }
            S *dst = T2 + (int64_t)k * sxy + col;
            if (full) {
                *reinterpret_cast<V *>(dst) = out;
            } else if (xin) {
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (i + q >= z.b.i0 && i + q < z.b.i1) dst[q] = lane_elem<S, VEC>(out, q);
            }
        }
        zm = zc;
        zc = zp;
        zp = zn;
        ci = cin;
        h = hn;
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
                       (C)a.rz, a.key, a.stochastic);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_step_boxes(int dtype, const StepArgs &a, const Box *b, int nb, hipStream_t s)
{
    if (dtype == IGG_F64) return run_boxes<double>(a, b, nb, s);
    if (dtype == IGG_F32) return run_boxes<float>(a, b, nb, s);
    return run_boxes<_Float16>(a, b, nb, s);
}

template <typename S, int VEC, int BX, int BYT>
static int run_zmarch(const StepArgs &a, const Box &b, hipStream_t s)
{
    using C = compute_t<S>;
    constexpr int TW = BX * VEC, BY = BYT - 2;
    ZTile z;
    z.b = b;
    z.nx = a.nx;
    z.ny = a.ny;
    z.xa = (b.i0 / VEC) * VEC;
    z.ntx = (b.i1 - z.xa + TW - 1) / TW;
    z.nty = (b.j1 - b.j0 + BY - 1) / BY;
    int depth = b.k1 - b.k0;
    int zc = env_int("IGG_ZCHUNK", 0);
    if (zc <= 0) {
        // enough work-groups to fill 256 CUs several times over, with long
        // enough marches that the two extra planes per chunk stay cheap
        int64_t cols = (int64_t)z.ntx * z.nty;
        int64_t want = 2048;
        int64_t chunks = (want + cols - 1) / cols;
        zc = (int)((depth + chunks - 1) / chunks);
        if (zc < 16) zc = 16;
    }
    if (zc > depth) zc = depth;
    z.zc = zc;
    z.remap = env_int("IGG_XCD_REMAP", 1);
    int64_t blocks = (int64_t)z.ntx * z.nty * ((depth + zc - 1) / zc);
    hipLaunchKernelGGL((k_step_zmarch<S, VEC, BX, BYT>), dim3((unsigned)blocks), dim3(BX * BYT), 0, s,
                       (S *)a.T2, (const S *)a.T, (const S *)a.Ci, z, (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz,
                       a.key, a.stochastic);
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

int launch_step_inner(int dtype, const StepArgs &a, const Box &b, hipStream_t s)
{
    if (dtype == IGG_F64) {
        if (vec_ok<double, 2>(a)) return run_zmarch<double, 2, 32, 16>(a, b, s);
        return run_zmarch<double, 1, 64, 8>(a, b, s);
    }
    if (dtype == IGG_F32) {
        if (vec_ok<float, 4>(a)) return run_zmarch<float, 4, 16, 16>(a, b, s);
        return run_zmarch<float, 1, 64, 8>(a, b, s);
    }
    if (vec_ok<_Float16, 8>(a)) return run_zmarch<_Float16, 8, 16, 16>(a, b, s);
    return run_zmarch<_Float16, 1, 64, 8>(a, b, s);
}

}  // namespace igg
