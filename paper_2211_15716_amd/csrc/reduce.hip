// reduce.hip -- FP64 reductions over a field (maximum(Ci) of Fig. 1, loss,
// conservation and dot-product sums).  Values are widened to FP64 before
// they are combined; rows are dealt to a fixed number of work-groups and
// combined in a fixed tree, so a call's bits do not vary between runs.
#include <mutex>
#include <string>

#include "host.hpp"

namespace igg {

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;

__device__ __forceinline__ double combine(int op, double x, double y)
{
    if (op == IGG_RED_MIN) return (x < y || x != x) ? x : y;
    if (op == IGG_RED_MAX || op == IGG_RED_MAX_ABS_DIFF || op == IGG_RED_MAX_ABS)
        return (x > y || x != x) ? x : y;
    return x + y;
}

__device__ __forceinline__ double identity(int op)
{
    if (op == IGG_RED_MIN) return __builtin_inf();
    if (op == IGG_RED_MAX || op == IGG_RED_MAX_ABS_DIFF || op == IGG_RED_MAX_ABS) return -__builtin_inf();
    return 0.0;
}

template <typename S>
__device__ __forceinline__ double term(int op, const S *a, const S *b, int64_t p)
{
    double x = (double)(compute_t<S>)a[p];
    switch (op) {
    case IGG_RED_SUM_RATIO: return x / (double)(compute_t<S>)b[p];
    case IGG_RED_HALF_SQDIFF: { double d = x - (double)(compute_t<S>)b[p]; return 0.5 * (d * d); }
    case IGG_RED_DOT: return x * (double)(compute_t<S>)b[p];
    case IGG_RED_MAX_ABS_DIFF: return __builtin_fabs(x - (double)(compute_t<S>)b[p]);
    case IGG_RED_MAX_ABS: return __builtin_fabs(x);
    default: return x;
    }
}

__device__ __forceinline__ double block_combine(int op, double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = combine(op, sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    return sh[0];
}

// Rows (j, k) of the region go to work-groups round-robin; each thread
// walks its row with a stride of the block size.
template <typename S>
__global__ void __launch_bounds__(RED_THREADS)
k_reduce(const S *__restrict__ a, const S *__restrict__ b, int op, int nx, int ny, int i0, int i1,
         int j0, int j1, int k0, int k1, double *__restrict__ part)
{
    __shared__ double sh[RED_THREADS];
    double acc = identity(op);
    const int64_t h = j1 - j0;
    const int64_t rows = h * (k1 - k0);
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int j = j0 + (int)(r % h), k = k0 + (int)(r / h);
        const int64_t base = (int64_t)k * nx * ny + (int64_t)j * nx;
        for (int i = i0 + threadIdx.x; i < i1; i += RED_THREADS) acc = combine(op, acc, term<S>(op, a, b, base + i));
    }
    double v = block_combine(op, acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// Combines the n partial results in `part` and writes the value to *result.
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_final(int op, int n, const double *__restrict__ part, double *__restrict__ result)
{
    __shared__ double sh[RED_THREADS];
    double acc = identity(op);
    for (int q = threadIdx.x; q < n; q += RED_THREADS) acc = combine(op, acc, part[q]);
    double v = block_combine(op, acc, sh);
    if (threadIdx.x == 0) *result = v;
}

// The two launches of a reduction: partial results of at most RED_BLOCKS
// work-groups into part[0..blocks), then their combination into *result.
template <typename S>
static int launch_two(int op, const igg_field &a, const igg_field *b, double *part, int part_cap, double *result,
                      hipStream_t s)
{
    const int nx = (int)a.size[0], ny = (int)a.size[1], nz = (int)a.size[2];
    const bool all = op == IGG_RED_MAX || op == IGG_RED_MIN;
    int i0 = all ? 0 : 1, i1 = all ? nx : nx - 1;
    int j0 = all ? 0 : 1, j1 = all ? ny : ny - 1;
    int k0 = all ? 0 : 1, k1 = all ? nz : nz - 1;
    int64_t rows = (int64_t)(j1 - j0) * (k1 - k0);
    int blocks = (int)(rows < RED_BLOCKS ? (rows < 1 ? 1 : rows) : RED_BLOCKS);
    if (blocks > part_cap)
        return fail(IGG_ERR_SIZE, "reduction needs " + std::to_string(blocks) + " partial results, the buffer holds " +
                                      std::to_string(part_cap));
    hipLaunchKernelGGL(k_reduce<S>, dim3(blocks), dim3(RED_THREADS), 0, s, (const S *)a.data,
                       b ? (const S *)b->data : (const S *)nullptr, op, nx, ny, i0, i1, j0, j1, k0, k1, part);
    IGG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, op, blocks, (const double *)part, result);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

static int launch_typed(int op, const igg_field &a, const igg_field *b, double *part, int part_cap, double *result,
                        hipStream_t s)
{
    if (b && b->dtype != a.dtype) return fail(IGG_ERR_DTYPE, "a and b must share one dtype");
    if (a.dtype == IGG_F64) return launch_two<double>(op, a, b, part, part_cap, result, s);
    if (a.dtype == IGG_F32) return launch_two<float>(op, a, b, part, part_cap, result, s);
    return launch_two<_Float16>(op, a, b, part, part_cap, result, s);
}

int launch_reduce(int op, const igg_field &a, const igg_field *b, double *out, hipStream_t s)
{
    Grid &g = grid();
    int rc;
    if ((rc = launch_typed(op, a, b, g.red_part, RED_BLOCKS, g.red_part + RED_BLOCKS, s))) return rc;
    IGG_HIP(hipMemcpyAsync(g.red_host, g.red_part + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
    IGG_HIP(hipStreamSynchronize(s));
    *out = g.red_host[0];
    return IGG_OK;
}

// ------------------------------------------------------- adjoint seed
// lam = a - b on the inner points (a alone without b, zero without a), zero
// on every halo point; with want_loss, the partial sums of 0.5*(a-b)^2 for
// k_reduce_final.  The inner rows are dealt to work-groups and walked by the
// threads exactly as k_reduce walks them for IGG_RED_HALF_SQDIFF, so the
// loss has the bits of that reduction.  The halo rows and columns are
// zeroed in a second walk.
template <typename S>
__global__ void __launch_bounds__(RED_THREADS)
k_seed(const S *__restrict__ a, const S *__restrict__ b, S *__restrict__ lam, int nx, int ny, int nz,
       double *__restrict__ part)
{
    using C = compute_t<S>;
    __shared__ double sh[RED_THREADS];
    double acc = 0.0;
    const int64_t h = ny - 2;
    const int64_t rows = h * (nz - 2);
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int j = 1 + (int)(r % h), k = 1 + (int)(r / h);
        const int64_t base = (int64_t)k * nx * ny + (int64_t)j * nx;
        for (int i = 1 + threadIdx.x; i < nx - 1; i += RED_THREADS) {
            const int64_t p = base + i;
            S v = S(0);
            if (a) {
                if (b) {
                    v = (S)((C)a[p] - (C)b[p]);
                    const double d = (double)(C)a[p] - (double)(C)b[p];
                    acc += 0.5 * (d * d);
                } else {
                    v = a[p];
                }
            }
            lam[p] = v;
        }
        if (threadIdx.x == 0) lam[base] = S(0);
        if (threadIdx.x == 1) lam[base + nx - 1] = S(0);
    }
    // halo rows: j = 0 and ny-1 of every plane, then every row of planes 0 and nz-1
    const int64_t hrows = 2 * (int64_t)nz + 2 * (int64_t)(ny - 2);
    for (int64_t r = blockIdx.x; r < hrows; r += gridDim.x) {
        int j, k;
        if (r < 2 * (int64_t)nz) {
            j = (r & 1) ? ny - 1 : 0;
            k = (int)(r >> 1);
        } else {
            const int64_t q = r - 2 * (int64_t)nz;
            j = 1 + (int)(q >> 1);
            k = (q & 1) ? nz - 1 : 0;
        }
        const int64_t base = (int64_t)k * nx * ny + (int64_t)j * nx;
        for (int i = threadIdx.x; i < nx; i += RED_THREADS) lam[base + i] = S(0);
    }
    if (part) {
        double v = block_combine(IGG_RED_HALF_SQDIFF, acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = v;
    }
}

int launch_seed(const igg_field *a, const igg_field *b, const igg_field &lam, double *loss, hipStream_t s)
{
    Grid &g = grid();
    const int nx = (int)lam.size[0], ny = (int)lam.size[1], nz = (int)lam.size[2];
    const int64_t rows = (int64_t)(ny - 2) * (nz - 2);
    const int blocks = (int)(rows < RED_BLOCKS ? (rows < 1 ? 1 : rows) : RED_BLOCKS);
    double *part = loss ? g.red_part : nullptr;
    if (lam.dtype == IGG_F64)
        hipLaunchKernelGGL(k_seed<double>, dim3(blocks), dim3(RED_THREADS), 0, s, a ? (const double *)a->data : nullptr,
                           b ? (const double *)b->data : nullptr, (double *)lam.data, nx, ny, nz, part);
    else if (lam.dtype == IGG_F32)
        hipLaunchKernelGGL(k_seed<float>, dim3(blocks), dim3(RED_THREADS), 0, s, a ? (const float *)a->data : nullptr,
                           b ? (const float *)b->data : nullptr, (float *)lam.data, nx, ny, nz, part);
    else
        hipLaunchKernelGGL(k_seed<_Float16>, dim3(blocks), dim3(RED_THREADS), 0, s,
                           a ? (const _Float16 *)a->data : nullptr, b ? (const _Float16 *)b->data : nullptr,
                           (_Float16 *)lam.data, nx, ny, nz, part);
    IGG_HIP(hipGetLastError());
    if (!loss) return IGG_OK;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, (int)IGG_RED_HALF_SQDIFF, blocks,
                       (const double *)g.red_part, g.red_part + RED_BLOCKS);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int read_reduce_result(double *out, hipStream_t s)
{
    Grid &g = grid();
    IGG_HIP(hipMemcpyAsync(g.red_host, g.red_part + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
    IGG_HIP(hipStreamSynchronize(s));
    *out = g.red_host[0];
    return IGG_OK;
}

// ----------------------------------------------------- without allocation
// Partial results of igg_reduce_noalloc: one array of 1024 doubles (8 KiB)
// per device, held until the process ends.  Every call writes the partial
// results it reads before reading them (same stream), so nothing needs
// clearing; calls that overlap in time on one device share the array and
// race.  Host code never uses its name as an address (on the host it is
// only a stand-in); it takes the device address that hipGetSymbolAddress
// returns for the current device, once per device.
constexpr int kNoallocScratch = 1024;
static __device__ __align__(256) double scratch[kNoallocScratch];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[IGG_MAX_DEVICES];

// The device address of `scratch` on the current device (looked up on the
// first call on that device).
static int scratch_on_current_device(double **ptr)
{
    int dev = -1;
    IGG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= IGG_MAX_DEVICES)
        return fail(IGG_ERR_ARG, "device index " + std::to_string(dev) + " above the library's limit");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        IGG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(IGG_ERR_HIP, "hipGetSymbolAddress returned a null address for the reduction scratch");
        g_scratch_ptr[dev] = (double *)p;
    }
    *ptr = g_scratch_ptr[dev];
    return IGG_OK;
}

int launch_reduce_noalloc(int op, const igg_field &a, const igg_field *b, double *out_dev, hipStream_t s)
{
    double *part = nullptr;
    int rc;
    if ((rc = scratch_on_current_device(&part))) return rc;
    return launch_typed(op, a, b, part, kNoallocScratch, out_dev, s);
}

}  // namespace igg
