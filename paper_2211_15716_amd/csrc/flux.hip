// flux.hip -- staggered-grid flux form of the diffusion step (Sec. 2 on the
// regular staggered grid): face fluxes q = -lam*grad(T), then the cell
// update T2 = T - dt*Ci*div(q), and the adjoint of that pair.
//
// Sizes: cells (nx,ny,nz); qx (nx+1,ny,nz), qy (nx,ny+1,nz), qz (nx,ny,nz+1).
// Face f of a dimension lies between cells f-1 and f; fluxes are computed on
// faces 1..n-1 of the inner rows of the other two dimensions.
#include "host.hpp"

namespace igg {

// Face field geometry for component d: extent of computed faces and strides.
struct FaceGeom {
    int nx, ny, nz;
};

template <typename C>
__device__ __forceinline__ bool face_index(int d, int64_t t, const FaceGeom &g, int &i, int &j, int &k)
{
    // computed faces: along d: 1..n_d-1 (n_d-1 faces); others: 1..n-2
    const int ex = d == 0 ? g.nx - 1 : g.nx - 2;
    const int ey = d == 1 ? g.ny - 1 : g.ny - 2;
    const int ez = d == 2 ? g.nz - 1 : g.nz - 2;
    if (t >= (int64_t)ex * ey * ez) return false;
    i = 1 + (int)(t % ex);
    int64_t r = t / ex;
    j = 1 + (int)(r % ey);
    k = 1 + (int)(r / ey);
    return true;
}

// q_d[f] = -lam*(V[f]-V[f-1])*rd for the cell field V (blockIdx.y = d).
// With mu_ci != null the cell field is mu = mu_ci .* V (the adjoint flux).
template <typename C>
__global__ void __launch_bounds__(256)
k_flux(C *__restrict__ qx, C *__restrict__ qy, C *__restrict__ qz, const C *__restrict__ V,
       const C *__restrict__ mu_ci, FaceGeom g, C lam, C rdx, C rdy, C rdz)
{
    const int d = blockIdx.y;
    int i, j, k;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!face_index<C>(d, t, g, i, j, k)) return;
    const int64_t cs = (d == 0) ? 1 : (d == 1) ? (int64_t)g.nx : (int64_t)g.nx * g.ny;
    const int64_t pc = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    C hi = V[pc], lo = V[pc - cs];
    if (mu_ci) {
        hi = mu_ci[pc] * hi;
        lo = mu_ci[pc - cs] * lo;
    }
    const C rd = d == 0 ? rdx : d == 1 ? rdy : rdz;
    const C v = -lam * ((hi - lo) * rd);
    if (d == 0)
        qx[i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k)] = v;
    else if (d == 1)
        qy[i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k)] = v;
    else
        qz[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] = v;
}

template <typename C>
__device__ __forceinline__ C divergence(const C *qx, const C *qy, const C *qz, int i, int j, int k,
                                        const FaceGeom &g, C rdx, C rdy, C rdz)
{
    const int64_t px = i + (int64_t)(g.nx + 1) * (j + (int64_t)g.ny * k);
    const int64_t py = i + (int64_t)g.nx * (j + (int64_t)(g.ny + 1) * k);
    const int64_t pz = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    const C dqx = (qx[px + 1] - qx[px]) * rdx;
    const C dqy = (qy[py + g.nx] - qy[py]) * rdy;
    const C dqz = (qz[pz + (int64_t)g.nx * g.ny] - qz[pz]) * rdz;
    return (dqx + dqy) + dqz;
}

// T2 = T - dt*Ci*div(q) on inner cells.
template <typename C>
__global__ void __launch_bounds__(256)
k_flux_update(C *__restrict__ T2, const C *__restrict__ T, const C *__restrict__ Ci, const C *__restrict__ qx,
              const C *__restrict__ qy, const C *__restrict__ qz, FaceGeom g, C dt, C rdx, C rdy, C rdz)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ex = g.nx - 2, ey = g.ny - 2;
    if (t >= (int64_t)ex * ey * (g.nz - 2)) return;
    const int i = 1 + (int)(t % ex);
    const int64_t r = t / ex;
    const int j = 1 + (int)(r % ey), k = 1 + (int)(r / ey);
    const int64_t p = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    const C div = divergence<C>(qx, qy, qz, i, j, k, g, rdx, rdy, rdz);
    T2[p] = fma_(-dt * Ci[p], div, T[p]);
}

// lam_n = lp - dt*div(p), gCi += -dt*lp*div(q) on inner cells.
template <typename C>
__global__ void __launch_bounds__(256)
k_flux_adj_update(C *__restrict__ lam_n, const C *__restrict__ lp, const C *__restrict__ px,
                  const C *__restrict__ py, const C *__restrict__ pz, const C *__restrict__ qx,
                  const C *__restrict__ qy, const C *__restrict__ qz, C *__restrict__ gCi, FaceGeom g, C dt,
                  C rdx, C rdy, C rdz)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ex = g.nx - 2, ey = g.ny - 2;
    if (t >= (int64_t)ex * ey * (g.nz - 2)) return;
    const int i = 1 + (int)(t % ex);
    const int64_t r = t / ex;
    const int j = 1 + (int)(r % ey), k = 1 + (int)(r / ey);
    const int64_t p = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    const C l = lp[p];
    lam_n[p] = fma_(-dt, divergence<C>(px, py, pz, i, j, k, g, rdx, rdy, rdz), l);
    gCi[p] = fma_(-dt * l, divergence<C>(qx, qy, qz, i, j, k, g, rdx, rdy, rdz), gCi[p]);
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename C>
static int run_flux(const FluxArgs &a, hipStream_t s)
{
    FaceGeom g{a.nx, a.ny, a.nz};
    int64_t most = (int64_t)(a.nx - 1) * (a.ny - 1) * (a.nz - 1);
    hipLaunchKernelGGL(k_flux<C>, dim3(blocks_for(most), 3), dim3(256), 0, s, (C *)a.qx, (C *)a.qy,
                       (C *)a.qz, (const C *)a.T, (const C *)nullptr, g, (C)a.lam, (C)a.rdx, (C)a.rdy,
                       (C)a.rdz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

template <typename C>
static int run_update(const FluxArgs &a, hipStream_t s)
{
    FaceGeom g{a.nx, a.ny, a.nz};
    int64_t n = (int64_t)(a.nx - 2) * (a.ny - 2) * (a.nz - 2);
    hipLaunchKernelGGL(k_flux_update<C>, dim3(blocks_for(n)), dim3(256), 0, s, (C *)a.T2, (const C *)a.T,
                       (const C *)a.Ci, (const C *)a.qx, (const C *)a.qy, (const C *)a.qz, g, (C)a.dt,
                       (C)a.rdx, (C)a.rdy, (C)a.rdz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

template <typename C>
static int run_adj(const FluxAdjArgs &a, hipStream_t s)
{
    FaceGeom g{a.nx, a.ny, a.nz};
    int64_t most = (int64_t)(a.nx - 1) * (a.ny - 1) * (a.nz - 1);
    // adjoint fluxes of mu = Ci .* lp
    hipLaunchKernelGGL(k_flux<C>, dim3(blocks_for(most), 3), dim3(256), 0, s, (C *)a.px, (C *)a.py,
                       (C *)a.pz, (const C *)a.lp, (const C *)a.Ci, g, (C)a.lam, (C)a.rdx, (C)a.rdy,
                       (C)a.rdz);
    IGG_HIP(hipGetLastError());
    int64_t n = (int64_t)(a.nx - 2) * (a.ny - 2) * (a.nz - 2);
    hipLaunchKernelGGL(k_flux_adj_update<C>, dim3(blocks_for(n)), dim3(256), 0, s, (C *)a.lam_n,
                       (const C *)a.lp, (const C *)a.px, (const C *)a.py, (const C *)a.pz, (const C *)a.qx,
                       (const C *)a.qy, (const C *)a.qz, (C *)a.gCi, g, (C)a.dt, (C)a.rdx, (C)a.rdy,
                       (C)a.rdz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_flux(int dtype, const FluxArgs &a, hipStream_t s)
{
    return dtype == IGG_F64 ? run_flux<double>(a, s) : run_flux<float>(a, s);
}

int launch_flux_update(int dtype, const FluxArgs &a, hipStream_t s)
{
    return dtype == IGG_F64 ? run_update<double>(a, s) : run_update<float>(a, s);
}

int launch_flux_adjoint(int dtype, const FluxAdjArgs &a, hipStream_t s)
{
    return dtype == IGG_F64 ? run_adj<double>(a, s) : run_adj<float>(a, s);
}

}  // namespace igg
