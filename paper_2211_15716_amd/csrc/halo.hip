// halo.hip -- halo update of the implicit global grid (Fig. 1 `update_halo!`,
// Sec. 2): per dimension x, y, z in turn, pack the two send planes of every
// field into contiguous buffers, exchange the buffers with the neighbours
// (on one process with a periodic dimension the neighbour on both sides is
// the process itself, so the exchange is a device copy between the send and
// receive buffers), and unpack the receive buffers into the halo planes.
#include "host.hpp"

namespace igg {

// One plane of one field: element (a, b) of the plane lives at
// base[plane*sd + a*sa + b*sb] and at buf[a + na*b].
struct PlaneDesc {
    unsigned char *base;
    unsigned char *buf;
    int64_t sd, sa, sb;
    int na, nb;
    int plane;
    int esz;
};

struct PlaneSet {
    PlaneDesc p[2 * IGG_MAX_FIELDS];
    int n;
};

template <typename E>
__device__ __forceinline__ void plane_copy(const PlaneDesc &d, int64_t e, bool to_buf)
{
    int a = (int)(e % d.na);
    int b = (int)(e / d.na);
    E *field = reinterpret_cast<E *>(d.base) + (int64_t)d.plane * d.sd + (int64_t)a * d.sa + (int64_t)b * d.sb;
    E *buf = reinterpret_cast<E *>(d.buf) + e;
    if (to_buf)
        *buf = *field;
    else
        *field = *buf;
}

// blockIdx.y selects the plane, x-threads walk its elements.
__global__ void __launch_bounds__(256) k_pack_unpack(PlaneSet ps, int to_buf)
{
    const PlaneDesc &d = ps.p[blockIdx.y];
    int64_t count = (int64_t)d.na * d.nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (d.esz == 8)
            plane_copy<uint64_t>(d, e, to_buf);
        else if (d.esz == 4)
            plane_copy<uint32_t>(d, e, to_buf);
        else
            plane_copy<uint16_t>(d, e, to_buf);
    }
}

// Exchange: copy `bytes` from src to dst for each pair (blockIdx.y); buffers
// are 256-byte aligned, so whole 16-byte words move as vectors.
struct CopySet {
    const unsigned char *src[2 * IGG_MAX_FIELDS];
    unsigned char *dst[2 * IGG_MAX_FIELDS];
    int64_t bytes[2 * IGG_MAX_FIELDS];
};

__global__ void __launch_bounds__(256) k_exchange(CopySet cs)
{
    const int q = blockIdx.y;
    const int64_t nvec = cs.bytes[q] / 16;
    const uint4 *s = reinterpret_cast<const uint4 *>(cs.src[q]);
    uint4 *d = reinterpret_cast<uint4 *>(cs.dst[q]);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = tid; e < nvec; e += stride) d[e] = s[e];
    const int64_t tail = cs.bytes[q] - nvec * 16;
    if (tid < tail) cs.dst[q][nvec * 16 + tid] = cs.src[q][nvec * 16 + tid];
}

static unsigned char *send_buf(Grid &g, int f, int side)
{
    return g.halo_buf + (size_t)(f * 2 + side) * g.halo_cap;
}

static unsigned char *recv_buf(Grid &g, int f, int side)
{
    return g.halo_buf + (size_t)(2 * IGG_MAX_FIELDS + f * 2 + side) * g.halo_cap;
}

static int grid_blocks(int64_t count)
{
    int64_t b = (count + 255) / 256;
    return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

int launch_halo(const igg_field *fl, int nf, hipStream_t s)
{
    Grid &g = grid();
    for (int d = 0; d < 3; ++d) {
        if (!g.periods[d]) continue;  // no neighbour in this dimension
        PlaneSet pk{}, up{};
        CopySet cs{};
        int64_t maxcount = 0;
        for (int f = 0; f < nf; ++f) {
            const igg_field &F = fl[f];
            const int64_t nx = F.size[0], ny = F.size[1], nz = F.size[2];
            const int nA = (int)F.size[d];
            const int olA = g.ol[d] + (nA - g.n[d]);
            PlaneDesc base{};
            base.base = (unsigned char *)F.data;
            base.esz = elem_bytes(F.dtype);
            if (d == 0) {
                base.sd = 1; base.na = (int)ny; base.sa = nx; base.nb = (int)nz; base.sb = nx * ny;
            } else if (d == 1) {
                base.sd = nx; base.na = (int)nx; base.sa = 1; base.nb = (int)nz; base.sb = nx * ny;
            } else {
                base.sd = nx * ny; base.na = (int)nx; base.sa = 1; base.nb = (int)ny; base.sb = nx;
            }
            int64_t count = (int64_t)base.na * base.nb;
            maxcount = count > maxcount ? count : maxcount;
            // pack: plane olA-1 -> send lo, plane nA-olA -> send hi
            PlaneDesc lo = base, hi = base;
            lo.plane = olA - 1; lo.buf = send_buf(g, f, 0);
            hi.plane = nA - olA; hi.buf = send_buf(g, f, 1);
            pk.p[pk.n++] = lo;
            pk.p[pk.n++] = hi;
            // exchange with the neighbours, here the process itself on both sides:
            // the upper neighbour's lo plane arrives in recv hi, the lower one's
            // hi plane in recv lo
            int64_t bytes = count * base.esz;
            cs.src[2 * f] = send_buf(g, f, 0); cs.dst[2 * f] = recv_buf(g, f, 1); cs.bytes[2 * f] = bytes;
            cs.src[2 * f + 1] = send_buf(g, f, 1); cs.dst[2 * f + 1] = recv_buf(g, f, 0); cs.bytes[2 * f + 1] = bytes;
            // unpack: recv lo -> plane 0, recv hi -> plane nA-1
            PlaneDesc ulo = base, uhi = base;
            ulo.plane = 0; ulo.buf = recv_buf(g, f, 0);
            uhi.plane = nA - 1; uhi.buf = recv_buf(g, f, 1);
            up.p[up.n++] = ulo;
            up.p[up.n++] = uhi;
        }
        dim3 grd(grid_blocks(maxcount), pk.n);
        hipLaunchKernelGGL(k_pack_unpack, grd, dim3(256), 0, s, pk, 1);
        IGG_HIP(hipGetLastError());
        int64_t maxvec = 0;
        for (int q = 0; q < 2 * nf; ++q) maxvec = cs.bytes[q] / 16 > maxvec ? cs.bytes[q] / 16 : maxvec;
        hipLaunchKernelGGL(k_exchange, dim3(grid_blocks(maxvec + 1), 2 * nf), dim3(256), 0, s, cs);
        IGG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pack_unpack, grd, dim3(256), 0, s, up, 0);
        IGG_HIP(hipGetLastError());
    }
    return IGG_OK;
}

}  // namespace igg
