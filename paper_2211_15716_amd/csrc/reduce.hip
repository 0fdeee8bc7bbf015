// reduce.hip -- FP64 reductions over a field (maximum(Ci) of Fig. 1, loss,
// conservation and dot-product sums).  Values are widened to FP64 before
// they are combined; rows are dealt to a fixed number of work-groups and
// combined in a fixed tree, so a call's bits do not vary between runs.
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

__global__ void __launch_bounds__(RED_THREADS) k_reduce_final(int op, int n, double *__restrict__ part)
{
    __shared__ double sh[RED_THREADS];
    double acc = identity(op);
    for (int q = threadIdx.x; q < n; q += RED_THREADS) acc = combine(op, acc, part[q]);
    double v = block_combine(op, acc, sh);
    if (threadIdx.x == 0) part[RED_BLOCKS] = v;
}

template <typename S>
static int run(int op, const igg_field &a, const igg_field *b, double *out, hipStream_t s)
{
    Grid &g = grid();
    const int nx = (int)a.size[0], ny = (int)a.size[1], nz = (int)a.size[2];
    const bool all = op == IGG_RED_MAX || op == IGG_RED_MIN;
    int i0 = all ? 0 : 1, i1 = all ? nx : nx - 1;
    int j0 = all ? 0 : 1, j1 = all ? ny : ny - 1;
    int k0 = all ? 0 : 1, k1 = all ? nz : nz - 1;
    int64_t rows = (int64_t)(j1 - j0) * (k1 - k0);
    int blocks = (int)(rows < RED_BLOCKS ? (rows < 1 ? 1 : rows) : RED_BLOCKS);
    hipLaunchKernelGGL(k_reduce<S>, dim3(blocks), dim3(RED_THREADS), 0, s, (const S *)a.data,
                       b ? (const S *)b->data : (const S *)nullptr, op, nx, ny, i0, i1, j0, j1, k0, k1,
                       g.red_part);
    IGG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, op, blocks, g.red_part);
    IGG_HIP(hipGetLastError());
    IGG_HIP(hipMemcpyAsync(g.red_host, g.red_part + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
    IGG_HIP(hipStreamSynchronize(s));
    *out = g.red_host[0];
    return IGG_OK;
}

int launch_reduce(int op, const igg_field &a, const igg_field *b, double *out, hipStream_t s)
{
    if (b && b->dtype != a.dtype) return fail(IGG_ERR_DTYPE, "a and b must share one dtype");
    if (a.dtype == IGG_F64) return run<double>(op, a, b, out, s);
    if (a.dtype == IGG_F32) return run<float>(op, a, b, out, s);
    return run<_Float16>(op, a, b, out, s);
}

}  // namespace igg
