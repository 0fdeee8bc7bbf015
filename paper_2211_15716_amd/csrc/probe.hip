// probe.hip -- streaming-bandwidth probe: the HBM rate a plain stream of a
// given read/write mix reaches on this device, the ceiling the stencil
// kernels are measured against beside the 8 TB/s peak.
//
// dst[w][i] = sum_r src[r][i], FP64, every array read or written exactly
// once, with non-temporal loads and stores (the accesses the stencil
// kernels use for the arrays they touch once).  Each thread moves one
// 16-byte vector per array, in work-groups of 256 threads over the whole
// array: on MI355X this streams faster than four vectors per thread (2R1W
// 6.40-6.46 against 6.24-6.32 TB/s), two (6.24), 512- or 1024-thread
// work-groups (5.83, 5.37 with four) or a grid-stride loop over fewer
// work-groups (5.82-5.98), so it is the ceiling the kernels are held to.
#include "host.hpp"

namespace igg {

typedef double d2v __attribute__((ext_vector_type(2)));

struct ProbeArgs {
    const d2v *s[4];
    d2v *d[4];
    int64_t n2;  // 16-byte vectors per array
};

constexpr int kProbeThreads = 256, kProbeUnroll = 1;

template <int NS, int ND>
__global__ void __launch_bounds__(kProbeThreads) k_stream_probe(ProbeArgs p)
{
    constexpr int64_t per_block = (int64_t)kProbeThreads * kProbeUnroll;
    const int64_t stride = (int64_t)gridDim.x * per_block;
    for (int64_t b = (int64_t)blockIdx.x * per_block + threadIdx.x; b < p.n2; b += stride) {
        d2v acc[kProbeUnroll];
#pragma unroll
        for (int q = 0; q < kProbeUnroll; ++q) acc[q] = d2v{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < NS; ++r)
#pragma unroll
            for (int q = 0; q < kProbeUnroll; ++q) {
                const int64_t i = b + (int64_t)q * kProbeThreads;
                if (i < p.n2) acc[q] += __builtin_nontemporal_load(p.s[r] + i);
            }
#pragma unroll
        for (int w = 0; w < ND; ++w)
#pragma unroll
            for (int q = 0; q < kProbeUnroll; ++q) {
                const int64_t i = b + (int64_t)q * kProbeThreads;
                if (i < p.n2) __builtin_nontemporal_store(acc[q], p.d[w] + i);
            }
    }
}

template <int NS>
static void launch_ns(int nd, const ProbeArgs &p, dim3 g, hipStream_t s)
{
    switch (nd) {
    case 1: hipLaunchKernelGGL((k_stream_probe<NS, 1>), g, dim3(kProbeThreads), 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_stream_probe<NS, 2>), g, dim3(kProbeThreads), 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_stream_probe<NS, 3>), g, dim3(kProbeThreads), 0, s, p); break;
    default: hipLaunchKernelGGL((k_stream_probe<NS, 4>), g, dim3(kProbeThreads), 0, s, p); break;
    }
}

}  // namespace igg

using namespace igg;

extern "C" int igg_stream_probe(const void *const *src, int nsrc, void *const *dst, int ndst, int64_t n,
                                void *stream)
{
    if (!src || !dst) return fail(IGG_ERR_ARG, "src or dst is null");
    if (nsrc < 1 || nsrc > 4 || ndst < 1 || ndst > 4)
        return fail(IGG_ERR_ARG, "nsrc and ndst must be in 1..4");
    if (n < 0 || n % 2) return fail(IGG_ERR_ARG, "n must be a non-negative even count of doubles");
    ProbeArgs p{};
    for (int r = 0; r < nsrc; ++r) {
        if (!src[r] || (uintptr_t)src[r] % 16) return fail(IGG_ERR_ARG, "src arrays must be 16-byte aligned");
        p.s[r] = (const d2v *)src[r];
    }
    for (int w = 0; w < ndst; ++w) {
        if (!dst[w] || (uintptr_t)dst[w] % 16) return fail(IGG_ERR_ARG, "dst arrays must be 16-byte aligned");
        p.d[w] = (d2v *)dst[w];
    }
    p.n2 = n / 2;
    if (p.n2 == 0) return IGG_OK;
    const int64_t per_block = (int64_t)kProbeThreads * kProbeUnroll;
    const int64_t blocks = std::min<int64_t>((p.n2 + per_block - 1) / per_block, (int64_t)1 << 20);
    const dim3 g((unsigned)blocks);
    hipStream_t s = (hipStream_t)stream;
    switch (nsrc) {
    case 1: launch_ns<1>(ndst, p, g, s); break;
    case 2: launch_ns<2>(ndst, p, g, s); break;
    case 3: launch_ns<3>(ndst, p, g, s); break;
    default: launch_ns<4>(ndst, p, g, s); break;
    }
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}
