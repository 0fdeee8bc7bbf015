// halo.hip -- halo update of the implicit global grid (Fig. 1 `update_halo!`,
// Sec. 2).  Neighbouring local grids share `ol` planes: my plane ol-1 is the
// last plane of my lower neighbour and my plane n-ol is the first plane of my
// upper neighbour.  For each dimension x, y, z in turn, the two planes of
// every field are packed into send buffers, exchanged (the lower neighbour
// receives plane ol-1 into the buffer that fills its last plane, the upper
// one plane n-ol into the buffer that fills its first plane), and unpacked.
// Dimensions go in order and planes are whole, so a later dimension carries
// the halo values an earlier one wrote, and edges and corners come out as
// images in every periodic dimension.
//
// The process holds every rank of the topology (one, or several virtual
// ranks as separate blocks on this device), so the exchange is a device copy
// from a rank's send buffer into its neighbour's receive buffer; a periodic
// dimension of one rank is its own neighbour on both sides.  One launch per
// dimension and rank runs all three phases: each thread packs its elements,
// exchanges them and unpacks them into the neighbour's halo.
#include "host.hpp"

namespace igg {

// One side of one field in one dimension.  Element (a, b) of a plane is at
// base[plane*sd + a*sa + b*sb] and at buf[a + na*b]; units are `esz` bytes
// (16 when whole rows move as 16-byte vectors).
struct HaloDesc {
    unsigned char *src_base;  // my field
    unsigned char *dst_base;  // the neighbour's field (mine on a periodic single rank)
    unsigned char *send;      // my send buffer for this side
    unsigned char *recv;      // the neighbour's receive buffer this side's data lands in
    int64_t sd, sa, sb;
    int na, nb;
    int src, dst;  // plane packed from, plane unpacked into
    int esz;
};

struct HaloSet {
    HaloDesc d[2 * IGG_MAX_FIELDS];
};

template <typename E>
__device__ __forceinline__ void halo_elem(const HaloDesc &d, int64_t e)
{
    const int a = (int)(e % d.na);
    const int b = (int)(e / d.na);
    const int64_t off = (int64_t)a * d.sa + (int64_t)b * d.sb;
    const E *A = reinterpret_cast<const E *>(d.src_base);
    E *B = reinterpret_cast<E *>(d.dst_base);
    E *send = reinterpret_cast<E *>(d.send);
    E *recv = reinterpret_cast<E *>(d.recv);
    send[e] = A[(int64_t)d.src * d.sd + off];  // pack
    recv[e] = send[e];                         // exchange (a device copy: the neighbour is on this GPU)
    B[(int64_t)d.dst * d.sd + off] = recv[e];  // unpack into the neighbour's halo
}

// blockIdx.y selects the (field, side); x-threads walk the plane.
__global__ void __launch_bounds__(256) k_halo_self(HaloSet hs)
{
    const HaloDesc &d = hs.d[blockIdx.y];
    const int64_t count = (int64_t)d.na * d.nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        switch (d.esz) {
        case 16: halo_elem<uint4>(d, e); break;
        case 8: halo_elem<uint64_t>(d, e); break;
        case 4: halo_elem<uint32_t>(d, e); break;
        default: halo_elem<uint16_t>(d, e); break;
        }
    }
}

// Rank r owns 4 * IGG_MAX_FIELDS planes: send buffers of (field, side), then
// receive buffers of (field, side); side 0 faces the lower neighbour.
static unsigned char *send_buf(Grid &g, int r, int f, int side)
{
    return g.halo_buf + ((size_t)r * 4 * IGG_MAX_FIELDS + f * 2 + side) * g.halo_cap;
}

static unsigned char *recv_buf(Grid &g, int r, int f, int side)
{
    return g.halo_buf + ((size_t)r * 4 * IGG_MAX_FIELDS + 2 * IGG_MAX_FIELDS + f * 2 + side) * g.halo_cap;
}

unsigned char *halo_send_plane(int r, int f, int side) { return send_buf(grid(), r, f, side); }

// Exchange and unpack of the planes the boundary-slab kernel packed, for a
// rank that is its own neighbour: the receive side of the exchange is the
// destination halo plane itself, so each element is copied once, from the
// send buffer into the field.  d[q] is plane q: element (a, b) of the
// packed plane (a fastest) goes to dst[a*sa + b*sb], units of esz bytes.
struct PlaneCopy {
    const unsigned char *src;
    unsigned char *dst;
    int64_t sa, sb;
    int na, nb;
    int esz;
};
struct PlaneCopySet {
    PlaneCopy d[4];
};

template <typename E>
__device__ __forceinline__ void copy_elem(const PlaneCopy &d, int64_t e)
{
    const int a = (int)(e % d.na);
    const int b = (int)(e / d.na);
    reinterpret_cast<E *>(d.dst)[(int64_t)a * d.sa + (int64_t)b * d.sb] = reinterpret_cast<const E *>(d.src)[e];
}

__global__ void __launch_bounds__(256) k_unpack_planes(PlaneCopySet ps)
{
    const PlaneCopy &d = ps.d[blockIdx.y];
    const int64_t count = (int64_t)d.na * d.nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        switch (d.esz) {
        case 16: copy_elem<uint4>(d, e); break;
        case 8: copy_elem<uint64_t>(d, e); break;
        case 4: copy_elem<uint32_t>(d, e); break;
        default: copy_elem<uint16_t>(d, e); break;
        }
    }
}

int launch_unpack_self(const igg_field &f, const SlabPack &pk, hipStream_t s)
{
    const int64_t nx = f.size[0], ny = f.size[1], nz = f.size[2];
    const int64_t e = elem_bytes(f.dtype);
    PlaneCopySet ps{};
    int64_t maxcount = 0;
    for (int d = 0; d < 2; ++d)
        for (int side = 0; side < 2; ++side) {
            PlaneCopy &c = ps.d[2 * d + side];
            c.esz = (int)e;
            c.src = (const unsigned char *)pk.send[d][side];
            c.na = (int)nx;
            c.sa = 1;
            if (d == 0) {  // y plane: a = x, b = z, into row j
                const int64_t j = side == 0 ? ny - 1 : 0;
                c.dst = (unsigned char *)f.data + j * nx * e;
                c.nb = (int)nz;
                c.sb = nx * ny;
            } else {  // z plane: a = x, b = y, into plane k
                const int64_t k = side == 0 ? nz - 1 : 0;
                c.dst = (unsigned char *)f.data + k * nx * ny * e;
                c.nb = (int)ny;
                c.sb = nx;
            }
            // whole rows as 16-byte vectors where the row length and base allow
            if ((nx * e) % 16 == 0 && ((uintptr_t)f.data % 16) == 0) {
                c.na = (int)(nx * e / 16);
                c.sb = c.sb * e / 16;
                c.esz = 16;
            }
            maxcount = std::max(maxcount, (int64_t)c.na * c.nb);
        }
    const int64_t b = (maxcount + 255) / 256;
    dim3 grd((unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 1024), 4);
    hipLaunchKernelGGL(k_unpack_planes, grd, dim3(256), 0, s, ps);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

// Gather form of the y and z halo update for a rank that is its own
// neighbour: plane q of the four (y side 0: j = ny-1, side 1: j = 0; z
// likewise) is filled point by point from the image of each point, the
// index map img(0) = n-ol, img(n-1) = ol-1, img(c) = c otherwise, applied in
// every dimension.  Images are inner points, which the step wrote, so the
// four planes are independent and one launch fills them.
struct SelfHalo {
    unsigned char *base;
    int nx, ny, nz;
    int ol[3];
    int esz;
};

__device__ __forceinline__ int self_img(int c, int n, int ol) { return c == 0 ? n - ol : (c == n - 1 ? ol - 1 : c); }

template <typename E>
__global__ void __launch_bounds__(256) k_halo_gather_yz(SelfHalo h)
{
    E *A = reinterpret_cast<E *>(h.base);
    const int q = blockIdx.y;  // 0, 1: y planes (ny-1, 0); 2, 3: z planes (nz-1, 0)
    const int64_t nx = h.nx, sxy = (int64_t)h.nx * h.ny;
    const int nb = q < 2 ? h.nz : h.ny;
    const int64_t count = nx * nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e % nx), b = (int)(e / nx);
        const int sa = self_img(a, h.nx, h.ol[0]);
        int64_t dst, src;
        if (q < 2) {
            const int j = q == 0 ? h.ny - 1 : 0;
            dst = (int64_t)b * sxy + (int64_t)j * nx + a;
            src = (int64_t)self_img(b, h.nz, h.ol[2]) * sxy + (int64_t)self_img(j, h.ny, h.ol[1]) * nx + sa;
        } else {
            const int k = q == 2 ? h.nz - 1 : 0;
            dst = (int64_t)k * sxy + (int64_t)b * nx + a;
            src = (int64_t)self_img(k, h.nz, h.ol[2]) * sxy + (int64_t)self_img(b, h.ny, h.ol[1]) * nx + sa;
        }
        A[dst] = A[src];
    }
}

int launch_halo_self_yz(const igg_field &f, hipStream_t s)
{
    Grid &g = grid();
    SelfHalo h{(unsigned char *)f.data, (int)f.size[0], (int)f.size[1], (int)f.size[2], {0, 0, 0},
               elem_bytes(f.dtype)};
    for (int d = 0; d < 3; ++d) h.ol[d] = g.ol[d] + (int)(f.size[d] - g.n[d]);
    const int64_t maxcount = (int64_t)h.nx * std::max(h.ny, h.nz);
    const int64_t b = (maxcount + 255) / 256;
    const dim3 grd((unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 1024), 4);
    if (h.esz == 8) hipLaunchKernelGGL(k_halo_gather_yz<uint64_t>, grd, dim3(256), 0, s, h);
    else if (h.esz == 4) hipLaunchKernelGGL(k_halo_gather_yz<uint32_t>, grd, dim3(256), 0, s, h);
    else hipLaunchKernelGGL(k_halo_gather_yz<uint16_t>, grd, dim3(256), 0, s, h);
    IGG_HIP(hipGetLastError());
    return IGG_OK;
}

int launch_halo(const igg_field *fl, int nf, hipStream_t s, int dims)
{
    Grid &g = grid();
    for (int d = 0; d < 3; ++d) {
        if (!((dims >> d) & 1)) continue;  // done elsewhere (fused into the step)
        for (int r = 0; r < g.nranks; ++r) {
            HaloSet hs{};
            int nd = 0;
            int64_t maxcount = 0;
            const int lo_nbr = rank_neighbor(r, d, 0), hi_nbr = rank_neighbor(r, d, 1);
            for (int f = 0; f < nf; ++f) {
                const igg_field &F = fl[(size_t)r * nf + f];
                const int64_t nx = F.size[0], ny = F.size[1], nz = F.size[2];
                const int nA = (int)F.size[d];
                const int olA = g.ol[d] + (nA - g.n[d]);
                HaloDesc base{};
                base.esz = elem_bytes(F.dtype);
                if (d == 0) {
                    base.sd = 1; base.na = (int)ny; base.sa = nx; base.nb = (int)nz; base.sb = nx * ny;
                } else if (d == 1) {
                    base.sd = nx; base.na = (int)nx; base.sa = 1; base.nb = (int)nz; base.sb = nx * ny;
                } else {
                    base.sd = nx * ny; base.na = (int)nx; base.sa = 1; base.nb = (int)ny; base.sb = nx;
                }
                // whole rows as 16-byte vectors where rows, strides and bases allow
                const int64_t e = base.esz;
                bool vec = base.sa == 1 && (base.na * e) % 16 == 0 && (base.sb * e) % 16 == 0 &&
                           (base.sd * e) % 16 == 0 && ((uintptr_t)F.data % 16) == 0;
                for (int q : {lo_nbr, hi_nbr})
                    if (q >= 0 && ((uintptr_t)fl[(size_t)q * nf + f].data % 16) != 0) vec = false;
                if (vec) {
                    base.na = (int)(base.na * e / 16);
                    base.sb = base.sb * e / 16;
                    base.sd = base.sd * e / 16;
                    base.esz = 16;
                }
                base.src_base = (unsigned char *)F.data;
                if (lo_nbr >= 0) {
                    // plane ol-1 becomes the lower neighbour's last plane
                    HaloDesc lo = base;
                    lo.dst_base = (unsigned char *)fl[(size_t)lo_nbr * nf + f].data;
                    lo.src = olA - 1;
                    lo.dst = nA - 1;
                    lo.send = send_buf(g, r, f, 0);
                    lo.recv = recv_buf(g, lo_nbr, f, 1);
                    hs.d[nd++] = lo;
                }
                if (hi_nbr >= 0) {
                    // plane n-ol becomes the upper neighbour's first plane
                    HaloDesc hi = base;
                    hi.dst_base = (unsigned char *)fl[(size_t)hi_nbr * nf + f].data;
                    hi.src = nA - olA;
                    hi.dst = 0;
                    hi.send = send_buf(g, r, f, 1);
                    hi.recv = recv_buf(g, hi_nbr, f, 0);
                    hs.d[nd++] = hi;
                }
                maxcount = std::max(maxcount, (int64_t)base.na * base.nb);
            }
            if (nd == 0) continue;  // no neighbour in this dimension
            int64_t b = (maxcount + 255) / 256;
            dim3 grd((unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 1024), nd);
            hipLaunchKernelGGL(k_halo_self, grd, dim3(256), 0, s, hs);
            IGG_HIP(hipGetLastError());
        }
    }
    return IGG_OK;
}

}  // namespace igg
