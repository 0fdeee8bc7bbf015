// device.hpp -- device-side building blocks shared by every kernel of the
// library: storage/compute types, the one stencil-point function, the
// counter-based hash and FP16 stochastic rounding, and the box descriptors
// the boundary-first schedule hands to kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace igg {

// ------------------------------------------------------------------ types
// Storage type S and the type C the arithmetic runs in.
template <typename S> struct Compute;
template <> struct Compute<double> { using type = double; };
template <> struct Compute<float> { using type = float; };
template <> struct Compute<_Float16> { using type = float; };
template <typename S> using compute_t = typename Compute<S>::type;

__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename C, typename S> __device__ __forceinline__ C widen(S v) { return static_cast<C>(v); }

// ------------------------------------------------------------ the stencil
// One point of the Fig. 1 step:
//   T2 = T + dt*lam*Ci*(d2x/dx^2 + d2y/dy^2 + d2z/dz^2),
//   d2x = (T[i+1]-T[i]) - (T[i]-T[i-1]).
// a = dt*lam and r* = 1/dd^2 are rounded once to C on the host.  Every
// kernel that computes a point calls this function with the same operands
// (the file is built with -ffp-contract=off and the fused operations are
// explicit), so a point's bits do not depend on which kernel computed it.
template <typename C>
__device__ __forceinline__ C diffuse(C c, C xm, C xp, C ym, C yp, C zm, C zp, C ci, C a, C rx,
                                     C ry, C rz)
{
    C d2x = (xp - c) - (c - xm);
    C d2y = (yp - c) - (c - ym);
    C d2z = (zp - c) - (c - zm);
    C lap = fma_(d2z, rz, fma_(d2y, ry, d2x * rx));
    return fma_(a * ci, lap, c);
}

// Second-difference sum sum_d d2_d(v)/dd^2 (used by the adjoint).
template <typename C>
__device__ __forceinline__ C laplace(C c, C xm, C xp, C ym, C yp, C zm, C zp, C rx, C ry, C rz)
{
    C d2x = (xp - c) - (c - xm);
    C d2y = (yp - c) - (c - ym);
    C d2z = (zp - c) - (c - zm);
    return fma_(d2z, rz, fma_(d2y, ry, d2x * rx));
}

// Face flux of the staggered form: q = -lam*(hi - lo)*rd for the cells on
// either side of the face, rd = 1/dd.
template <typename C>
__device__ __forceinline__ C face_flux(C hi, C lo, C lam, C rd)
{
    return -lam * ((hi - lo) * rd);
}

// Divergence of a cell's six face fluxes (lower l, upper u per dimension).
template <typename C>
__device__ __forceinline__ C flux_div(C qxl, C qxu, C qyl, C qyu, C qzl, C qzu, C rdx, C rdy, C rdz)
{
    return ((qxu - qxl) * rdx + (qyu - qyl) * rdy) + (qzu - qzl) * rdz;
}

// ------------------------------------------------------------------ hash
// PCG hash of Jarzynski and Olano, "Hash Functions for GPU Rendering",
// JCGT 9(3), 2020: one LCG step of O'Neill's PCG followed by its RXS-M-XS
// output permutation; a bijection of 32-bit words.
// pcg_hash(v) = pcg_permute(v * kPcgMul + kPcgInc).
constexpr uint32_t kPcgMul = 747796405u, kPcgInc = 2891336453u;

__host__ __device__ __forceinline__ uint32_t pcg_permute(uint32_t state)
{
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

__host__ __device__ __forceinline__ uint32_t pcg_hash(uint32_t v) { return pcg_permute(v * kPcgMul + kPcgInc); }

// Key of one plane k for the key of a (seed, counter) pair.
__device__ __forceinline__ uint32_t plane_key(uint32_t key, int k) { return pcg_hash(key + (uint32_t)k); }

// Global origin of a block for the FP16 stochastic-rounding hash: the point
// (i, j, k) of the block is hashed as (i + ox, j + oy, k + oz) in a global
// index space gnx points wide, so every decomposition rounds a point alike.
// In a periodic dimension global indices g and g + p* (p* = dims*(n-ol), the
// period) are one physical point, held by overlapping planes of the same or
// neighbouring blocks; the index is taken modulo the period (0: not
// periodic), so every copy of a point draws the same random bits.
struct SrOrigin {
    int ox, oy, oz, gnx;
    int px, py, pz;
    int gnh;  // (gnx + 1) / 2: pairs of points per global row
};

__device__ __forceinline__ int sr_wrap(int g, int p) { return (p && g >= p) ? g - p : g; }

// Key of plane k of a block for the key of a (seed, counter) pair.
__device__ __forceinline__ uint32_t sr_plane_key(uint32_t key, int k, const SrOrigin &so)
{
    return plane_key(key, sr_wrap(k + so.oz, so.pz));
}

// Random bits of point (i, j) of a block's plane with key pk.  One 32-bit
// hash serves the two points 2m and 2m+1 of a global row (indices taken
// modulo the period): the even point takes its high 16 bits, the odd point
// its low 16 bits, each as the top half of its 32-bit word (FP16 stochastic
// rounding uses the top 13 bits of the word in the normal range, the top 16
// for subnormals).  The hashed word is pk + n for the pair's index n in the
// plane (mod 2^32), so its first multiply splits as n*kPcgMul, fixed for a
// point through a z-march, plus pk*kPcgMul, one per plane.  A kernel holding
// both points of a pair hashes once for the two (sr_point_bits2).
__device__ __forceinline__ uint32_t sr_pair_index(int gi, int gj, const SrOrigin &so)
{
    return (uint32_t)(gi >> 1) + (uint32_t)so.gnh * (uint32_t)gj;
}

__device__ __forceinline__ uint32_t sr_pair_word(uint32_t pk, int gi, int gj, const SrOrigin &so)
{
    return pcg_hash(pk + sr_pair_index(gi, gj, so));
}

__device__ __forceinline__ uint32_t sr_half(uint32_t w, int gi) { return (gi & 1) ? (w << 16) : w; }

__device__ __forceinline__ uint32_t sr_point_bits(uint32_t pk, int i, int j, const SrOrigin &so)
{
    const int gi = sr_wrap(i + so.ox, so.px);
    return sr_half(sr_pair_word(pk, gi, sr_wrap(j + so.oy, so.py), so), gi);
}

// The bits of points (i, j) and (i+1, j): one hash when they are one pair
// (even global index and no period wrap between them), else two.
__device__ __forceinline__ void sr_point_bits2(uint32_t pk, int i, int j, const SrOrigin &so, uint32_t &r0,
                                               uint32_t &r1)
{
    const int gi0 = sr_wrap(i + so.ox, so.px), gi1 = sr_wrap(i + 1 + so.ox, so.px);
    const int gj = sr_wrap(j + so.oy, so.py);
    const uint32_t w0 = sr_pair_word(pk, gi0, gj, so);
    if ((gi0 & 1) == 0 && gi1 == gi0 + 1) {
        r0 = w0;
        r1 = w0 << 16;
    } else {
        r0 = sr_half(w0, gi0);
        r1 = sr_half(sr_pair_word(pk, gi1, gj, so), gi1);
    }
}

// ---------------------------------------------------- FP16 stores
// Unbiased stochastic rounding of a float to FP16 with the random word w:
// x is rounded up to the next FP16 value with probability equal to its
// distance from the lower one divided by their spacing.  In the FP16 normal
// range that is adding the top 13 bits of w (uniform) below the FP16 ulp to
// the magnitude and truncating (an FP16 value has 13 fewer fraction bits
// than a float: exact probabilities); gfx950 does exactly this in one
// instruction (v_cvt_sr_f16_f32 takes the top 13 bits of its random
// operand and gives the bits of the integer form, (bits(x) + (w >> 19)) &
// ~0x1FFF: the GPU tests check every stored value of a step against that
// form computed on the host).  In the
// subnormal range the spacing is 2^-24 and the fraction is compared with
// the top 16 bits of w as a uniform in [0, 1) (probabilities to 2^-16).
// Values already representable in FP16 are returned unchanged.
__device__ __forceinline__ _Float16 round_sr(float x, uint32_t w)
{
    float ax = __builtin_fabsf(x);
    if (ax < 65504.0f && ax >= 6.103515625e-05f) {  // FP16 normal range (2^-14 and up)
        // the instruction writes one half of its destination and keeps the
        // other; w's register (dead after this) serves as that destination
        typedef _Float16 H2 __attribute__((ext_vector_type(2)));
        H2 v = __builtin_bit_cast(H2, w);
        v = __builtin_amdgcn_cvt_sr_f16_f32(v, x, w, false);
        return v[0];
    }
    if (!(ax < 65504.0f)) return (_Float16)x;  // overflow, inf, nan
    float s = ax * 16777216.0f;  // exact: multiples of 2^-24 become integers
    float f = __builtin_floorf(s);
    float u = (float)(w >> 16) * (1.0f / 65536.0f);
    float m = (u < s - f) ? f + 1.0f : f;
    return (_Float16)__builtin_copysignf(m * 5.9604644775390625e-08f, x);
}

// Whether all four values lie in the FP16 normal range, where the gfx950
// instruction rounds them as round_sr does: the smallest magnitude at least
// 2^-14 and the sum of magnitudes below 65504 (the sum is at least the
// largest magnitude, and is not below 65504 for an infinity or a NaN).
__device__ __forceinline__ bool sr_normal4(const float (&v)[4])
{
    const float a0 = __builtin_fabsf(v[0]), a1 = __builtin_fabsf(v[1]), a2 = __builtin_fabsf(v[2]),
                a3 = __builtin_fabsf(v[3]);
    const float lo = __builtin_fminf(__builtin_fminf(a0, a1), __builtin_fminf(a2, a3));
    const float sum = (a0 + a1) + (a2 + a3);
    return lo >= 6.103515625e-05f && sum < 65504.0f;
}

template <typename S> struct Store {
    template <typename C> __device__ __forceinline__ static S put(C v, uint32_t, int) { return (S)v; }
};
template <> struct Store<_Float16> {
    __device__ __forceinline__ static _Float16 put(float v, uint32_t r, int stochastic)
    {
        // v is an FP32 value, rounded once to FP16 here.  The empty asm keeps
        // the compiler from folding the conversion into the multiply-add that
        // produced v (v_fma_mixlo/hi_f16 round the exact result to FP16 once,
        // which can differ from rounding it to FP32 first): without it, some
        // points of some kernels got the folded form and a point's bits
        // depended on which kernel computed it.
        __asm__("" : "+v"(v));
        return stochastic ? round_sr(v, r) : (_Float16)v;
    }
};

// ------------------------------------------------------- buffer access
// Loads and stores of a whole vector type T (2, 4, 8 or 16 bytes) at a byte
// offset from a buffer descriptor's base (AUX = 2: non-temporal).  A
// descriptor per array and plane lives in scalar registers, so a kernel
// addresses its lanes with 32-bit offsets instead of 64-bit pointers.
template <typename T, int AUX>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    constexpr int B = sizeof(T);
    static_assert(B == 2 || B == 4 || B == 8 || B == 16, "buffer access of 2, 4, 8 or 16 bytes");
    if constexpr (B == 2)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, AUX));
    else if constexpr (B == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
    else if constexpr (B == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX));
}
template <typename T, int AUX>
__device__ __forceinline__ void buf_store(const T &v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    constexpr int B = sizeof(T);
    static_assert(B == 2 || B == 4 || B == 8 || B == 16, "buffer access of 2, 4, 8 or 16 bytes");
    using U8 = unsigned int __attribute__((ext_vector_type(2)));
    using U16 = unsigned int __attribute__((ext_vector_type(4)));
    if constexpr (B == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, 0, AUX);
    else if constexpr (B == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, AUX);
    else if constexpr (B == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U8, v), r, off, 0, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U16, v), r, off, 0, AUX);
}

// A descriptor for the bytes [p, p + bytes) (bytes below 2^31).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}

// ------------------------------------------------------------------ boxes
// Half-open index box [i0,i1) x [j0,j1) x [k0,k1).
struct Box {
    int i0, i1, j0, j1, k0, k1;
};

// Up to 6 boxes walked by one launch.  Each box's rows (j,k) are cut into
// segments of `lpr` lanes (a power of two, >= the box width up to 64), so a
// 15-point-wide slab packs four rows into one 64-lane wavefront.
struct BoxSet {
    Box b[6];
    int lpr_log2[6];
    int nseg_x[6];   // segments per row
    int64_t first[7];  // first thread of each box (prefix sum), first[n] = total
    int n;
};

// Map a global thread index to a point of a box set; returns false for
// threads past the end or lanes past a row segment's end.
__device__ __forceinline__ bool boxset_point(const BoxSet &bs, int64_t t, int &i, int &j, int &k)
{
    int b = 0;
#pragma unroll
    for (int q = 1; q < 6; ++q)
        if (q < bs.n && t >= bs.first[q]) b = q;
    if (t >= bs.first[bs.n]) return false;
    const Box &bx = bs.b[b];
    int64_t local = t - bs.first[b];
    int lane = (int)(local & ((1 << bs.lpr_log2[b]) - 1));
    int64_t seg = local >> bs.lpr_log2[b];
    int sx = (int)(seg % bs.nseg_x[b]);
    int64_t row = seg / bs.nseg_x[b];
    int h = bx.j1 - bx.j0;
    i = bx.i0 + (sx << bs.lpr_log2[b]) + lane;
    j = bx.j0 + (int)(row % h);
    k = bx.k0 + (int)(row / h);
    return i < bx.i1;
}

// ------------------------------------------------------------ XCD mapping
// Work-groups of one launch are handed to the 8 XCDs (each with its own L2)
// in turn: group g runs on XCD g % 8.  Renumber them so each XCD receives
// one contiguous range of logical tiles; tiles that share halo rows then
// share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t g, int64_t n)
{
    const int64_t X = 8;
    int64_t q = n / X, r = n % X;
    int64_t x = g % X, slot = g / X;
    return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

}  // namespace igg
