// adjoint.hip -- transposed diffusion step.
//
// The forward step is T_{n+1} = T_n + a*Ci.*(L T_n) on the inner points
// (a = dt*lam, L = sum_d d2_d/dd^2, symmetric on the periodic grid).  Given
// lp = dLoss/dT_{n+1} with a valid halo, one adjoint step computes
//   lam_n = lp + a*L(mu),  mu = Ci.*lp        (mu formed on the fly at the
//                                               six neighbours)
//   gCi  += a*lp.*(L T_n)
// on the inner points.  k_adj_boxes is the one-thread-per-point form used
// for the boundary slabs; k_adj_zmarch marches z like the forward kernel,
// keeping lp, Ci and T_n of planes k-1, k, k+1 in registers and staging mu
// and T_n of plane k in LDS for the x and y neighbours.
#include <stdlib.h>

#include "host.hpp"

namespace igg {

template <typename C>
__device__ __forceinline__ void adjoint_point(C l, C lapmu, C lapT, C a, C &lam_n, C &g)
{
    lam_n = fma_(a, lapmu, l);
    g = fma_(a * l, lapT, g);
}

template <typename C>
__global__ void __launch_bounds__(256)
k_adj_boxes(C *__restrict__ lam_n, const C *__restrict__ lp, const C *__restrict__ Tn,
            const C *__restrict__ Ci, C *__restrict__ gCi, BoxSet bs, int nx, int ny, C a, C rx, C ry,
            C rz)
{
    int i, j, k;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!boxset_point(bs, t, i, j, k)) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t p = i + sy * j + sz * k;
    auto mu = [&](int64_t q) { return Ci[q] * lp[q]; };
    C lapmu = laplace<C>(mu(p), mu(p - 1), mu(p + 1), mu(p - sy), mu(p + sy), mu(p - sz), mu(p + sz), rx,
                         ry, rz);
    C lapT = laplace<C>(Tn[p], Tn[p - 1], Tn[p + 1], Tn[p - sy], Tn[p + sy], Tn[p - sz], Tn[p + sz], rx, ry,
                        rz);
    C ln, g = gCi[p];
    adjoint_point<C>(lp[p], lapmu, lapT, a, ln, g);
    lam_n[p] = ln;
    gCi[p] = g;
}

struct AdjTile {
    Box b;
    int nx, ny;
    int xa;
    int ntx, nty;
    int zc;
    int remap;
};

// BX x BYT threads, one point per thread; rows 0 and BYT-1 load y-halos.
template <typename C, int BX, int BYT>
__global__ void __launch_bounds__(BX *BYT)
k_adj_zmarch(C *__restrict__ lam_n, const C *__restrict__ lp, const C *__restrict__ Tn,
             const C *__restrict__ Ci, C *__restrict__ gCi, AdjTile z, C a, C rx, C ry, C rz)
{
    constexpr int BY = BYT - 2, LW = BX + 2;
    __shared__ C smu[2][BYT][LW];
    __shared__ C sT[2][BYT][LW];
    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    const int64_t g = z.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int bx = (int)(g % z.ntx);
    const int64_t rest = g / z.ntx;
    const int by = (int)(rest % z.nty);
    const int bz = (int)(rest / z.nty);
    const int nx = z.nx, ny = z.ny;
    const int64_t sxy = (int64_t)nx * ny;
    const int x0 = z.xa + bx * BX;
    const int i = x0 + tx;
    const int j = z.b.j0 + by * BY + ty - 1;
    const int jc = j < 0 ? 0 : (j > ny - 1 ? ny - 1 : j);
    const bool xin = i < nx;
    const bool crow = ty >= 1 && ty <= BY && j < z.b.j1 && i >= z.b.i0 && i < z.b.i1;
    const int kb = z.b.k0 + bz * z.zc;
    const int ke = (kb + z.zc < z.b.k1) ? kb + z.zc : z.b.k1;
    const int64_t col = (int64_t)jc * nx + i;
    const bool hl = tx == 0 && x0 >= 1;
    const bool hr = tx == BX - 1 && x0 + BX < nx;
    const bool own_h = hl || hr;
    const int64_t colh = (int64_t)jc * nx + (tx == 0 ? x0 - 1 : x0 + BX);

    auto ld = [&](const C *A, int k, int64_t c, bool ok) -> C { return ok ? A[(int64_t)k * sxy + c] : C(0); };

    // mu and T of planes k-1, k, k+1 for this column
    C mm = ld(Ci, kb - 1, col, xin) * ld(lp, kb - 1, col, xin);
    C lc = ld(lp, kb, col, xin);
    C mc = ld(Ci, kb, col, xin) * lc;
    C lpn = ld(lp, kb + 1, col, xin);
    C mp = ld(Ci, kb + 1, col, xin) * lpn;
    C tm = ld(Tn, kb - 1, col, xin), tc = ld(Tn, kb, col, xin), tp = ld(Tn, kb + 1, col, xin);
    C hmu = own_h ? ld(Ci, kb, colh, true) * ld(lp, kb, colh, true) : C(0);
    C hT = ld(Tn, kb, colh, own_h);

    for (int k = kb; k < ke; ++k) {
        const int buf = (k - kb) & 1;
        const bool more = k + 1 < ke;
        C ln2 = 0, mn = 0, tn = 0, hmu_n = 0, hT_n = 0;
        if (more) {
            ln2 = ld(lp, k + 2, col, xin);
            mn = ld(Ci, k + 2, col, xin) * ln2;
            tn = ld(Tn, k + 2, col, xin);
            if (own_h) {
                hmu_n = ld(Ci, k + 1, colh, true) * ld(lp, k + 1, colh, true);
                hT_n = ld(Tn, k + 1, colh, true);
            }
        }
        smu[buf][ty][1 + tx] = mc;
        sT[buf][ty][1 + tx] = tc;
        if (own_h) {
            smu[buf][ty][tx == 0 ? 0 : LW - 1] = hmu;
            sT[buf][ty][tx == 0 ? 0 : LW - 1] = hT;
        }
        __syncthreads();
        if (crow) {
            const int c = 1 + tx;
            C lapmu = laplace<C>(mc, smu[buf][ty][c - 1], smu[buf][ty][c + 1], smu[buf][ty - 1][c],
                                 smu[buf][ty + 1][c], mm, mp, rx, ry, rz);
            C lapT = laplace<C>(tc, sT[buf][ty][c - 1], sT[buf][ty][c + 1], sT[buf][ty - 1][c],
                                sT[buf][ty + 1][c], tm, tp, rx, ry, rz);
            const int64_t p = (int64_t)k * sxy + col;
            C ln, gg = gCi[p];
            adjoint_point<C>(lc, lapmu, lapT, a, ln, gg);
            lam_n[p] = ln;
            gCi[p] = gg;
        }
        mm = mc;
        mc = mp;
        mp = mn;
        lc = lpn;
        lpn = ln2;
        tm = tc;
        tc = tp;
        tp = tn;
        hmu = hmu_n;
        hT = hT_n;
    }
}

static int env_int(const char *name, int dflt)
{
    const char *s = getenv(name);
    return (s && *s) ? atoi(s) : dflt;
}

template <typename C>
static int run_boxes(const AdjArgs &a, const Box *b, int nb, hipStream_t s)
{
    BoxSet bs = make_boxset(b, nb);
    int64_t threads = bs.first[nb];
    if (threads == 0) return IGG_OK;
    hipLaunchKernelGGL(k_adj_boxes<C>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       (C *)a.lam_n, (const C *)a.lp, (const C *)a.Tn, (const C *)a.Ci, (C *)a.gCi, bs,
                       a.nx, a.ny, (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_adjoint_boxes(int dtype, const AdjArgs &a, const Box *b, int nb, hipStream_t s)
{
    return dtype == IGG_F64 ? run_boxes<double>(a, b, nb, s) : run_boxes<float>(a, b, nb, s);
}

template <typename C, int BX, int BYT>
static int run_zmarch(const AdjArgs &a, const Box &b, hipStream_t s)
{
    constexpr int BY = BYT - 2;
    AdjTile z;
    z.b = b;
    z.nx = a.nx;
    z.ny = a.ny;
    z.xa = b.i0;
    z.ntx = (b.i1 - b.i0 + BX - 1) / BX;
    z.nty = (b.j1 - b.j0 + BY - 1) / BY;
    int depth = b.k1 - b.k0;
    int zc = env_int("IGG_ADJ_ZCHUNK", 0);
    if (zc <= 0) {
        int64_t cols = (int64_t)z.ntx * z.nty;
        int64_t chunks = (2048 + cols - 1) / cols;
        zc = (int)((depth + chunks - 1) / chunks);
        if (zc < 16) zc = 16;
    }
    if (zc > depth) zc = depth;
    z.zc = zc;
    z.remap = env_int("IGG_XCD_REMAP", 1);
    int64_t blocks = (int64_t)z.ntx * z.nty * ((depth + zc - 1) / zc);
    hipLaunchKernelGGL((k_adj_zmarch<C, BX, BYT>), dim3((unsigned)blocks), dim3(BX * BYT), 0, s,
                       (C *)a.lam_n, (const C *)a.lp, (const C *)a.Tn, (const C *)a.Ci, (C *)a.gCi, z,
                       (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_adjoint_inner(int dtype, const AdjArgs &a, const Box &b, hipStream_t s)
{
    return dtype == IGG_F64 ? run_zmarch<double, 64, 8>(a, b, s) : run_zmarch<float, 64, 8>(a, b, s);
}

}  // namespace igg
