// adjoint.hip -- transposed diffusion step, for the Laplacian form and the
// staggered flux form.
//
// The forward step is T_{n+1} = T_n + a*Ci.*(L T_n) on the inner points
// (a = dt*lam, L = sum_d d2_d/dd^2, symmetric on the periodic grid).  Given
// lp = dLoss/dT_{n+1} with a valid halo, one adjoint step computes
//   lam_n = lp + a*L(mu),  mu = Ci.*lp        (mu formed on the fly at the
//                                               six neighbours)
//   gCi  += a*lp.*(L T_n)
// on the inner points.  k_adj_boxes is the one-thread-per-point form used
// for the boundary slabs; k_adj_zmarch marches z with the forward kernel's
// tiling, keeping lp, mu and T_n of planes k-1, k, k+1 in registers and
// staging mu and T_n of plane k in LDS for the x and y neighbours.
#include <stdlib.h>

#include "host.hpp"

namespace igg {

template <typename C>
__device__ __forceinline__ void adjoint_point(C l, C lapmu, C lapT, C a, C &lam_n, C &g)
{
    lam_n = fma_(a, lapmu, l);
    g = fma_(a * l, lapT, g);
}

// One cell of the adjoint from mu = Ci.*lp and T_n at the cell and its six
// neighbours.  FORM 0, the Laplacian step (a = dt*lam, r = 1/dd^2):
//   lam_n = lp + a*L(mu),  gCi += a*lp*L(T_n).
// FORM 1, the staggered flux form (a = dt, r = 1/dd, lamf = lam), with the
// face fluxes p = -lam*grad(mu) and q = -lam*grad(T_n) formed on the fly:
//   lam_n = lp - dt*div(p),  gCi += -dt*lp*div(q).
template <typename C, int FORM>
__device__ __forceinline__ void adj_cell(C l, C m0, C mxm, C mxp, C mym, C myp, C mzm, C mzp, C t0, C txm,
                                         C txp, C tym, C typ, C tzm, C tzp, C a, C rx, C ry, C rz, C lamf,
                                         C &ln, C &g)
{
    if constexpr (FORM == 0) {
        const C lapmu = laplace<C>(m0, mxm, mxp, mym, myp, mzm, mzp, rx, ry, rz);
        const C lapT = laplace<C>(t0, txm, txp, tym, typ, tzm, tzp, rx, ry, rz);
        adjoint_point<C>(l, lapmu, lapT, a, ln, g);
    } else {
        const C divp = flux_div<C>(face_flux<C>(m0, mxm, lamf, rx), face_flux<C>(mxp, m0, lamf, rx),
                                   face_flux<C>(m0, mym, lamf, ry), face_flux<C>(myp, m0, lamf, ry),
                                   face_flux<C>(m0, mzm, lamf, rz), face_flux<C>(mzp, m0, lamf, rz), rx, ry, rz);
        const C divq = flux_div<C>(face_flux<C>(t0, txm, lamf, rx), face_flux<C>(txp, t0, lamf, rx),
                                   face_flux<C>(t0, tym, lamf, ry), face_flux<C>(typ, t0, lamf, ry),
                                   face_flux<C>(t0, tzm, lamf, rz), face_flux<C>(tzp, t0, lamf, rz), rx, ry, rz);
        ln = fma_(-a, divp, l);
        g = fma_(-a * l, divq, g);
    }
}

// The y/z halo rows of row j at plane k under YZImg: every (jj, kk) other
// than (j, k) with jj in {j, ny-1 if j = jl, 0 if j = jh} and kk in {k,
// nz-1 if k = kl, 0 if k = kh} (with n = ol+1 one row is the image of both
// halo rows).  f(jj, kk) is called for each.
template <typename F>
__device__ __forceinline__ void yz_images(const YZImg &yz, int j, int k, F &&f)
{
    if (j != yz.jl && j != yz.jh && k != yz.kl && k != yz.kh) return;
    const int js[3] = {j, j == yz.jl ? yz.ny - 1 : -1, j == yz.jh ? 0 : -1};
    const int ks[3] = {k, k == yz.kl ? yz.nz - 1 : -1, k == yz.kh ? 0 : -1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if ((a | b) && js[a] >= 0 && ks[b] >= 0) f(js[a], ks[b]);
}

template <typename C, int FORM>
__global__ void __launch_bounds__(256)
k_adj_boxes(C *__restrict__ lam_n, const C *__restrict__ lp, const C *__restrict__ Tn,
            const C *__restrict__ Ci, C *__restrict__ gCi, BoxSet bs, int nx, int ny, C a, C rx, C ry,
            C rz, C lamf, XHalo xh, YZImg yz)
{
    int i, j, k;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!boxset_point(bs, t, i, j, k)) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t p = i + sy * j + sz * k;
    auto mu = [&](int64_t q) { return Ci[q] * lp[q]; };
    C ln, g = gCi[p];
    adj_cell<C, FORM>(lp[p], mu(p), mu(p - 1), mu(p + 1), mu(p - sy), mu(p + sy), mu(p - sz), mu(p + sz), Tn[p],
                      Tn[p - 1], Tn[p + 1], Tn[p - sy], Tn[p + sy], Tn[p - sz], Tn[p + sz], a, rx, ry, rz, lamf,
                      ln, g);
    lam_n[p] = ln;
    gCi[p] = g;
    // x exchange of lam_n fused into the store
    if (xh.on_lo && i == xh.lo) lam_n[p - i + nx - 1 + xh.d_lo] = ln;
    if (xh.on_hi && i == xh.hi) lam_n[p - i + xh.d_hi] = ln;
    // y/z halo planes whose image is this point, each with its x exchange
    if (yz.on)
        yz_images(yz, j, k, [&](int jj, int kk) {
            const int64_t q0 = sz * kk + sy * jj;
            lam_n[q0 + i] = ln;
            if (xh.on_lo && i == xh.lo) lam_n[q0 + nx - 1 + xh.d_lo] = ln;
            if (xh.on_hi && i == xh.hi) lam_n[q0 + xh.d_hi] = ln;
        });
}

struct AdjTile {
    Box b;
    int nx, ny;
    int xa;
    int ntx, nty;
    int zc;
    int remap;
    int rblock;  // mode 2: x-rows of tiles per block dealt to one XCD
    XHalo xh;
    YZImg yz;
};

template <typename C, int VEC> struct AVec {
    typedef C type __attribute__((ext_vector_type(VEC)));
};
template <typename C> struct AVec<C, 1> {
    typedef C type;
};
template <typename C, int VEC>
__device__ __forceinline__ C el(const typename AVec<C, VEC>::type &v, int q)
{
    if constexpr (VEC == 1)
        return v;
    else
        return v[q];
}
// element q of a vector for a q known only at run time
template <typename C, int VEC>
__device__ __forceinline__ C el_dyn(const typename AVec<C, VEC>::type &v, int q)
{
    C x = el<C, VEC>(v, 0);
#pragma unroll
    for (int p = 1; p < VEC; ++p)
        if (q == p) x = el<C, VEC>(v, p);
    return x;
}
template <typename C, int VEC>
__device__ __forceinline__ void set_el(typename AVec<C, VEC>::type &v, int q, C x)
{
    if constexpr (VEC == 1)
        v = x;
    else
        v[q] = x;
}

// BX x TY threads, RY rows of VEC points per thread (the forward kernel's
// tiling).  mu = Ci .* lp and T_n of plane k are staged in two
// double-buffered LDS tiles; lp, mu and T_n of planes k-1..k+1 (k+2 in
// flight) sit in registers.  gCi is read and written once per point and
// lam_n written once: non-temporal.  The products mu of the planes in
// flight are formed when the queue rotates, after the plane's arithmetic,
// so the loads are not waited for inside the plane (256^3: 3.5% faster).
template <typename C, int VEC, int BX, int TY, int RY, int FORM, int WAVES>
__global__ void __launch_bounds__(BX *TY) __attribute__((amdgpu_waves_per_eu(WAVES)))
k_adj_zmarch(C *__restrict__ lam_n, const C *__restrict__ lp, const C *__restrict__ Tn,
             const C *__restrict__ Ci, C *__restrict__ gCi, AdjTile z, C a, C rx, C ry, C rz, C lamf)
{
    using V = typename AVec<C, VEC>::type;
    static_assert(BX == 64, "a wave holds one thread row (the y/z image stores rely on it)");
    constexpr int TW = BX * VEC, TH = TY * RY, LH = TH + 2, LW = TW + 2;
    __shared__ C smu[2][LH][LW];
    __shared__ C sT[2][LH][LW];
    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    int64_t g = blockIdx.x;
    if (z.remap == 2) {  // blocks of rblock x-rows of tiles dealt to the XCDs in turn
        const int64_t ntx0 = z.ntx, B = z.rblock, P = gridDim.x / ntx0, P8 = P / (8 * B) * (8 * B);
        if (g < ntx0 * P8) {
            const int64_t x = g % 8, slot = g / 8, q = slot / ntx0;
            g = slot % ntx0 + ntx0 * (((q / B) * 8 + x) * B + q % B);
        }
    }
    const int bx = (int)(g % z.ntx);
    const int64_t rest = g / z.ntx;
    const int by = (int)(rest % z.nty);
    const int bz = (int)(rest / z.nty);
    const int nx = z.nx, ny = z.ny;
    const int64_t sxy = (int64_t)nx * ny;
    const int x0 = z.xa + bx * TW;
    const int i = x0 + tx * VEC;
    const bool xin = i < nx;
    const int jb = z.b.j0 + by * TH;
    const int kb = z.b.k0 + bz * z.zc;
    const int ke = (kb + z.zc < z.b.k1) ? kb + z.zc : z.b.k1;
    int64_t col[RY];
    bool crow[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int j = jb + ty * RY + r;
        col[r] = (int64_t)(j > ny - 1 ? ny - 1 : j) * nx + i;
        crow[r] = j < z.b.j1;
    }
    const bool hy = ty == 0 || ty == TY - 1;
    const int jh = (ty == 0) ? jb - 1 : (jb + TH > ny - 1 ? ny - 1 : jb + TH);
    const int64_t colhy = (int64_t)jh * nx + i;
    const int hyrow = (ty == 0) ? 0 : LH - 1;
    const bool own_h = (tx == 0 && x0 >= 1) || (tx == BX - 1 && x0 + TW < nx);
    const int xh = (tx == 0) ? x0 - 1 : x0 + TW;
    const int hcol = (tx == 0) ? 0 : LW - 1;

    // loads through a buffer descriptor per array and plane (scalar
    // registers) with 32-bit byte offsets in the plane (the launcher keeps
    // planes below 2 GiB): no 64-bit address registers per lane, which
    // leaves room under the 128-register cap for the deferred products below
    const int64_t pb = sxy * (int64_t)sizeof(C);
    auto rs = [&](const C *A, int k) { return buf_rsrc(A + (int64_t)k * sxy, pb); };
    auto ld = [&](const C *A, int k, int64_t c) -> V {
        V v{};
        if (xin) v = buf_load<V, 0>(rs(A, k), (uint32_t)(c * (int64_t)sizeof(C)));
        return v;
    };
    auto ld_nt = [&](const C *A, int k, int64_t c) -> V {
        V v{};
        if (xin) v = buf_load<V, 2>(rs(A, k), (uint32_t)(c * (int64_t)sizeof(C)));
        return v;
    };
    auto lds1 = [&](const C *A, int k, int64_t c) -> C { return buf_load<C, 0>(rs(A, k), (uint32_t)(c * (int64_t)sizeof(C))); };
    auto mul = [](V x, V y) -> V {
        V out;
#pragma unroll
        for (int q = 0; q < VEC; ++q) set_el<C, VEC>(out, q, el<C, VEC>(x, q) * el<C, VEC>(y, q));
        return out;
    };

    V mm[RY], mc[RY], mp[RY], tm[RY], tc[RY], tp[RY], lc[RY], lq[RY], gc[RY];
    C hmu[RY], hT[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        mm[r] = mul(ld(Ci, kb - 1, col[r]), ld(lp, kb - 1, col[r]));
        lc[r] = ld(lp, kb, col[r]);
        mc[r] = mul(ld(Ci, kb, col[r]), lc[r]);
        lq[r] = ld(lp, kb + 1, col[r]);
        mp[r] = mul(ld(Ci, kb + 1, col[r]), lq[r]);
        tm[r] = ld(Tn, kb - 1, col[r]);
        tc[r] = ld(Tn, kb, col[r]);
        tp[r] = ld(Tn, kb + 1, col[r]);
        gc[r] = crow[r] ? ld_nt(gCi, kb, col[r]) : V{};
        const int64_t ph = col[r] - i + xh;
        hmu[r] = own_h ? lds1(Ci, kb, ph) * lds1(lp, kb, ph) : C(0);
        hT[r] = own_h ? lds1(Tn, kb, ph) : C(0);
    }
    V ymu = hy ? mul(ld(Ci, kb, colhy), ld(lp, kb, colhy)) : V{};
    V yT = hy ? ld(Tn, kb, colhy) : V{};

    for (int k = kb; k < ke; ++k) {
        const int buf = (k - kb) & 1;
        const bool more = k + 1 < ke;
        // loads for the next planes, consumed one iteration later (Ci and
        // lp raw: their products are formed at the rotation below)
        V cn[RY], tn[RY], ln2[RY], gn[RY], yc_n{}, yl_n{}, yT_n{};
        C hc_n[RY], hl_n[RY], hT_n[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            ln2[r] = more ? ld(lp, k + 2, col[r]) : V{};
            cn[r] = more ? ld(Ci, k + 2, col[r]) : V{};
            tn[r] = more ? ld(Tn, k + 2, col[r]) : V{};
            gn[r] = (more && crow[r]) ? ld_nt(gCi, k + 1, col[r]) : V{};
            const int64_t ph = col[r] - i + xh;
            hc_n[r] = (more && own_h) ? lds1(Ci, k + 1, ph) : C(0);
            hl_n[r] = (more && own_h) ? lds1(lp, k + 1, ph) : C(0);
            hT_n[r] = (more && own_h) ? lds1(Tn, k + 1, ph) : C(0);
        }
        if (more && hy) {
            yc_n = ld(Ci, k + 1, colhy);
            yl_n = ld(lp, k + 1, colhy);
            yT_n = ld(Tn, k + 1, colhy);
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int lr = 1 + ty * RY + r;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                smu[buf][lr][1 + tx * VEC + q] = el<C, VEC>(mc[r], q);
                sT[buf][lr][1 + tx * VEC + q] = el<C, VEC>(tc[r], q);
            }
            if (own_h) {
                smu[buf][lr][hcol] = hmu[r];
                sT[buf][lr][hcol] = hT[r];
            }
        }
        if (hy) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                smu[buf][hyrow][1 + tx * VEC + q] = el<C, VEC>(ymu, q);
                sT[buf][hyrow][1 + tx * VEC + q] = el<C, VEC>(yT, q);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!crow[r]) continue;
            const int lr = 1 + ty * RY + r;
            V lo, go;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int lc_ = 1 + tx * VEC + q;
                const C m0 = el<C, VEC>(mc[r], q), t0 = el<C, VEC>(tc[r], q);
                const C mxm = (q == 0) ? smu[buf][lr][lc_ - 1] : el<C, VEC>(mc[r], q - 1);
                const C mxp = (q == VEC - 1) ? smu[buf][lr][lc_ + 1] : el<C, VEC>(mc[r], q + 1);
                const C mym = (r == 0) ? smu[buf][lr - 1][lc_] : el<C, VEC>(mc[r - 1], q);
                const C myp = (r == RY - 1) ? smu[buf][lr + 1][lc_] : el<C, VEC>(mc[r + 1], q);
                const C txm = (q == 0) ? sT[buf][lr][lc_ - 1] : el<C, VEC>(tc[r], q - 1);
                const C txp = (q == VEC - 1) ? sT[buf][lr][lc_ + 1] : el<C, VEC>(tc[r], q + 1);
                const C tym = (r == 0) ? sT[buf][lr - 1][lc_] : el<C, VEC>(tc[r - 1], q);
                const C typ = (r == RY - 1) ? sT[buf][lr + 1][lc_] : el<C, VEC>(tc[r + 1], q);
                C ln, gg = el<C, VEC>(gc[r], q);
                adj_cell<C, FORM>(el<C, VEC>(lc[r], q), m0, mxm, mxp, mym, myp, el<C, VEC>(mm[r], q),
                                  el<C, VEC>(mp[r], q), t0, txm, txp, tym, typ, el<C, VEC>(tm[r], q),
                                  el<C, VEC>(tp[r], q), a, rx, ry, rz, lamf, ln, gg);
                set_el<C, VEC>(lo, q, ln);
                set_el<C, VEC>(go, q, gg);
            }
            const int64_t p = (int64_t)k * sxy + col[r];
            if (xin && i >= z.b.i0 && i + VEC <= z.b.i1) {
                const uint32_t ob = (uint32_t)(col[r] * (int64_t)sizeof(C));
                buf_store<V, 2>(lo, rs(lam_n, k), ob);
                buf_store<V, 2>(go, rs(gCi, k), ob);
            } else if (xin) {
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (i + q >= z.b.i0 && i + q < z.b.i1) {
                        lam_n[p + q] = el<C, VEC>(lo, q);
                        gCi[p + q] = el<C, VEC>(go, q);
                    }
            }
            // x exchange of lam_n fused into the store
            if (z.xh.on_lo && xin && i <= z.xh.lo && i + VEC > z.xh.lo && z.xh.lo >= z.b.i0 && z.xh.lo < z.b.i1)
                lam_n[p - i + nx - 1 + z.xh.d_lo] = el_dyn<C, VEC>(lo, z.xh.lo - i);
            if (z.xh.on_hi && xin && i <= z.xh.hi && i + VEC > z.xh.hi && z.xh.hi >= z.b.i0 && z.xh.hi < z.b.i1)
                lam_n[p - i + z.xh.d_hi] = el_dyn<C, VEC>(lo, z.xh.hi - i);
            // y/z halo rows whose image is this row, each with its x exchange
            // (a wave holds one row, BX being 64: the row index is the same
            // in every lane, and the branch is taken by whole waves)
            if (z.yz.on && xin)
                yz_images(z.yz, __builtin_amdgcn_readfirstlane(jb + ty * RY + r), k, [&](int jj, int kk) {
                    C *row = lam_n + (int64_t)kk * sxy + (int64_t)jj * nx;
#pragma unroll
                    for (int q = 0; q < VEC; ++q)
                        if (i + q >= z.b.i0 && i + q < z.b.i1) row[i + q] = el<C, VEC>(lo, q);
                    if (z.xh.on_lo && i <= z.xh.lo && i + VEC > z.xh.lo && z.xh.lo >= z.b.i0 && z.xh.lo < z.b.i1)
                        row[nx - 1 + z.xh.d_lo] = el_dyn<C, VEC>(lo, z.xh.lo - i);
                    if (z.xh.on_hi && i <= z.xh.hi && i + VEC > z.xh.hi && z.xh.hi >= z.b.i0 && z.xh.hi < z.b.i1)
                        row[z.xh.d_hi] = el_dyn<C, VEC>(lo, z.xh.hi - i);
                });
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            mm[r] = mc[r];
            mc[r] = mp[r];
            mp[r] = mul(cn[r], ln2[r]);
            lc[r] = lq[r];
            lq[r] = ln2[r];
            tm[r] = tc[r];
            tc[r] = tp[r];
            tp[r] = tn[r];
            gc[r] = gn[r];
            hmu[r] = hc_n[r] * hl_n[r];
            hT[r] = hT_n[r];
        }
        ymu = mul(yc_n, yl_n);
        yT = yT_n;
    }
}

static int env_int(const char *name, int dflt)
{
    const char *s = getenv(name);
    return (s && *s) ? atoi(s) : dflt;
}

template <typename C, int FORM>
static int run_boxes(const AdjArgs &a, const Box *b, int nb, hipStream_t s)
{
    BoxSet bs = make_boxset(b, nb);
    int64_t threads = bs.first[nb];
    if (threads == 0) return IGG_OK;
    hipLaunchKernelGGL((k_adj_boxes<C, FORM>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       (C *)a.lam_n, (const C *)a.lp, (const C *)a.Tn, (const C *)a.Ci, (C *)a.gCi, bs,
                       a.nx, a.ny, (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz, (C)a.lamf, a.xh, a.yz);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_adjoint_boxes(int dtype, const AdjArgs &a, const Box *b, int nb, hipStream_t s)
{
    if (a.form == 1) return dtype == IGG_F64 ? run_boxes<double, 1>(a, b, nb, s) : run_boxes<float, 1>(a, b, nb, s);
    return dtype == IGG_F64 ? run_boxes<double, 0>(a, b, nb, s) : run_boxes<float, 0>(a, b, nb, s);
}

template <typename C, int VEC, int BX, int TY, int RY, int FORM, int WAVES = 1>
static int run_zmarch(const AdjArgs &a, const Box &b, hipStream_t s)
{
    constexpr int TW = BX * VEC, TH = TY * RY;
    AdjTile z;
    z.b = b;
    z.nx = a.nx;
    z.ny = a.ny;
    z.xa = (b.i0 / VEC) * VEC;
    z.ntx = (b.i1 - z.xa + TW - 1) / TW;
    z.nty = (b.j1 - b.j0 + TH - 1) / TH;
    int depth = b.k1 - b.k0;
    int zc = env_int("IGG_ADJ_ZCHUNK", 0);
    // chunks of at most 8 planes: 2% faster than 16 at 256^3 (FP64, 4-row
    // tiles) and 3% at 512^3
    if (zc < 1) zc = zchunk_for_groups((int64_t)z.ntx * z.nty, depth, 8);
    z.zc = zc;
    z.remap = env_int("IGG_ADJ_REMAP", 2);
    // blocks of 4 x-rows of tiles per XCD, so y-neighbour tiles share an
    // L2: the fastest block at 256^3 and 768^3 (by 2-6% over 1, 8, 16 and
    // 24); at 512^3 blocks of 16 are 4% faster
    z.rblock = std::max(1, env_int("IGG_ADJ_XCD_BLOCK", 4));
    z.xh = a.xh;
    z.yz = a.yz;
    int64_t blocks = (int64_t)z.ntx * z.nty * ((depth + zc - 1) / zc);
    if (blocks == 0) return IGG_OK;
    hipLaunchKernelGGL((k_adj_zmarch<C, VEC, BX, TY, RY, FORM, WAVES>), dim3((unsigned)blocks), dim3(BX * TY), 0, s,
                       (C *)a.lam_n, (const C *)a.lp, (const C *)a.Tn, (const C *)a.Ci, (C *)a.gCi, z,
                       (C)a.a, (C)a.rx, (C)a.ry, (C)a.rz, (C)a.lamf);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

static bool aligned(const void *p, int bytes) { return ((uintptr_t)p % (uintptr_t)bytes) == 0; }

template <typename C, int VEC = 2>
static bool vec2_ok(const AdjArgs &a)
{
    const int vb = VEC * (int)sizeof(C);
    return a.nx % VEC == 0 && aligned(a.lam_n, vb) && aligned(a.lp, vb) && aligned(a.Tn, vb) &&
           aligned(a.Ci, vb) && aligned(a.gCi, vb);
}

// 1 KB tile rows of 4 rows, 256 threads, one row per thread (the two
// staged fields need many registers), 16-byte loads: FP64 128 points per
// row (10% faster than 512-byte rows of 16 at 256^3 and 512^3 on MI355X;
// two rows per thread need 206 registers; since the products of the planes
// in flight moved to the rotation, 16-row tiles of 1024 threads pay at
// 512^3, see below),
// FP32 256 points (24% faster than 8-byte loads on 512-byte rows at 512^3
// and 768^3).  Narrower vectors, then one point per lane, where the row
// length or alignment does not allow 16-byte loads.  The FP64 kernel is
// held to 128 registers, which fits without spills and lets 4 waves share
// each SIMD instead of 3: the kernel is partly latency-bound, and that made
// it 11% faster at 256^3 and 5% at 512^3 (unsplit; both forms).
template <int FORM>
static int adjoint_inner(int dtype, const AdjArgs &a, const Box &b, hipStream_t s)
{
    if (dtype == IGG_F64)
    {
        if (!vec2_ok<double>(a)) return run_zmarch<double, 1, 64, 8, 2, FORM>(a, b, s);
        const int waves = env_int("IGG_ADJ_WAVES", 4);
        if (waves != 4) return run_zmarch<double, 2, 64, 4, 1, FORM>(a, b, s);
        // regions of 2^26 points and more: 16-row tiles over 1024 threads
        // (512^3: 4-10% faster than 4 rows on three boxes; 384^3 and 256^3
        // keep 4 rows, equal or faster there)
        if (box_count(b) >= ((int64_t)1 << 26)) return run_zmarch<double, 2, 64, 16, 1, FORM, 4>(a, b, s);
        return run_zmarch<double, 2, 64, 4, 1, FORM, 4>(a, b, s);
    }
    if (vec2_ok<float, 4>(a)) return run_zmarch<float, 4, 64, 4, 1, FORM>(a, b, s);
    return vec2_ok<float>(a) ? run_zmarch<float, 2, 64, 8, 1, FORM>(a, b, s)
                             : run_zmarch<float, 1, 64, 8, 2, FORM>(a, b, s);
}

int launch_adjoint_inner(int dtype, const AdjArgs &a, const Box &b, hipStream_t s)
{
    // the z-march kernel addresses a plane with 32-bit offsets (2 GiB at most)
    const int64_t plane = (int64_t)a.nx * a.ny * (dtype == IGG_F64 ? 8 : 4);
    if (box_count(b) < zmarch_min_points() || plane >= ((int64_t)1 << 31))
        return launch_adjoint_boxes(dtype, a, &b, 1, s);
    return a.form == 1 ? adjoint_inner<1>(dtype, a, b, s) : adjoint_inner<0>(dtype, a, b, s);
}

}  // namespace igg
