/*
 * igg.h -- C ABI of the MI355X explicit 3-D diffusion library with implicit
 * global grid halo updates.
 *
 * Paper: S. Omlin, L. Raess, I. Utkin, "Distributed Parallelization of xPU
 * Stencil Computations in Julia", JuliaCon proceedings (arXiv 2211.15716).
 * The API follows the paper's three-function model (Sec. 2: create the
 * implicit global grid, update halos, finalize it), the global-size queries
 * used by the Fig. 1 listing, and the listing's `step!` kernel fused with the
 * halo update under boundary-first overlap (Fig. 1, `@hide_communication`).
 * Beside the paper it offers an adjoint of the step, FP32 and FP16-storage
 * forms and the staggered flux form of the same update.
 *
 * General rules
 *   - Every function returns an int status: IGG_OK (0) or a negative
 *     IGG_ERR_* code; igg_last_error() returns a message for the calling
 *     thread's last failure.
 *   - Fields are dense device arrays in HBM, x fastest: element (i,j,k) is
 *     at data[i + nx*(j + ny*k)] (a torch tensor of shape (nz,ny,nx)).
 *     The caller owns every field.  Indices 0 and n-1 of each dimension are
 *     halo planes; 1..n-2 are the inner points.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous and ordered with respect to it, except igg_reduce and
 *     diffusion_dt, which synchronise it to return a host value.
 *   - Argument checks all run on the host before any HIP call, so a call
 *     with invalid arguments fails without touching the GPU.
 *   - One grid exists per process (the paper's calls take no handle).  The
 *     library owns its halo buffers, one helper stream and its events; they
 *     are created on the current HIP device at the first call that needs the
 *     GPU, and released by igg_finalize_global_grid.  Calls that overlap in
 *     time (from several host threads, or on unordered streams) race on the
 *     shared halo buffers and are not supported.
 *   - Environment variables choose schedules and launch shapes only; no
 *     setting changes a result bit.  Read by igg_init_global_grid:
 *     IGG_SCHEDULE (0, 1, 2 or 3: see diffusion_step; unset = by size and
 *     type), IGG_X_EXCHANGE ("halo": x slabs and an x pass of the halo
 *     update instead of the x exchange stored by the step kernels),
 *     IGG_SLAB_PACK (0: the y and z halo planes move in a separate halo
 *     pass; 1: the slab kernel packs them into send buffers and one copy
 *     unpacks them; 2, the default: it stores them straight into the halo
 *     planes), IGG_ZMARCH_MIN_POINTS (smallest region for the z-march
 *     kernels), IGG_TEST_DELAY ("side:N", "inner:N" or "halo:N": a wait of
 *     N rounds of about 3.4 us put into one stream of the split schedule,
 *     for tests that the streams are ordered by events, not by timing).
 *     Read at each launch (tuning): IGG_FP64_MIDTILE_MAX_POINTS (regions
 *     below it take the FP64 step tile of 2 rows per thread and 16 rows,
 *     larger ones 4 rows per thread and 32 rows), IGG_ZCHUNK, IGG_XCD_REMAP,
 *     IGG_XCD_BLOCK, IGG_XSLAB_ZCHUNK, IGG_XSLAB_REMAP, IGG_SLAB_MARCH,
 *     IGG_ADJ_ZCHUNK, IGG_ADJ_REMAP, IGG_ADJ_XCD_BLOCK, IGG_ADJ_WAVES,
 *     IGG_FLUX_ZCHUNK, IGG_FLUX_REMAP.
 */
#ifndef IGG_MI355X_H
#define IGG_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define IGG_OK 0
#define IGG_ERR_STATE (-1) /* grid not initialised, or initialised twice      */
#define IGG_ERR_ARG (-2)   /* null pointer or out-of-range scalar argument    */
#define IGG_ERR_SIZE (-3)  /* field sizes do not fit the grid or each other   */
#define IGG_ERR_DTYPE (-4) /* unsupported or mixed element types              */
#define IGG_ERR_ALIAS (-5) /* an output field shares memory with an input     */
#define IGG_ERR_HIP (-6)   /* a HIP runtime call failed (message has details) */

/* element types */
#define IGG_F64 0 /* double: FP64 storage and arithmetic                      */
#define IGG_F32 1 /* float: FP32 storage and arithmetic                       */
#define IGG_F16 2 /* _Float16 storage, FP32 arithmetic                        */

/* rounding of FP16 stores */
#define IGG_ROUND_NEAREST 0    /* round to nearest even                        */
#define IGG_ROUND_STOCHASTIC 1 /* unbiased stochastic rounding (see below)     */

/* reductions (igg_reduce) */
#define IGG_RED_MAX 0          /* max over ALL points of a (maximum(Ci))       */
#define IGG_RED_MIN 1          /* min over ALL points of a                      */
#define IGG_RED_SUM 2          /* sum of a over inner points                    */
#define IGG_RED_SUM_RATIO 3    /* sum of a/b over inner points                  */
#define IGG_RED_HALF_SQDIFF 4  /* 0.5*sum (a-b)^2 over inner points (the loss)  */
#define IGG_RED_DOT 5          /* sum a*b over inner points                     */
#define IGG_RED_MAX_ABS_DIFF 6 /* max |a-b| over inner points                   */
#define IGG_RED_MAX_ABS 7      /* max |a| over inner points                     */

#define IGG_MAX_FIELDS 8 /* fields per igg_update_halo call */
#define IGG_MAX_RANKS 64 /* virtual ranks of one grid (product of dims) */

/* A field: a device pointer, its element type and its size per dimension. */
typedef struct igg_field {
    void *data;       /* device pointer, 16-byte alignment gives vector loads */
    int32_t dtype;    /* IGG_F64, IGG_F32 or IGG_F16                          */
    int32_t reserved; /* must be 0                                            */
    int64_t size[3];  /* nx, ny, nz of this field                             */
} igg_field;

/* Rounding of FP16 stores.  Stochastic rounding draws its random bits from a
 * counter-based hash of (seed, counter, point index), so the same step with
 * the same counter rounds identically however the work is split; exactly
 * representable values are never moved.  Pass a new counter every step. */
typedef struct igg_rounding {
    int32_t mode;     /* IGG_ROUND_NEAREST or IGG_ROUND_STOCHASTIC */
    int32_t reserved; /* must be 0 */
    uint64_t seed;
    uint64_t counter;
} igg_rounding;

/* ------------------------------------------------------- grid (Sec. 2) */

/* Create the implicit global grid (Sec. 2; Fig. 1 `init_global_grid`).
 *   nx, ny, nz   local grid size; each must exceed the overlap (n >= ol+1).
 *   dims         ranks per dimension, NULL or 0 = 1.  A product P > 1 (at
 *                most IGG_MAX_RANKS) makes this process hold all P ranks of
 *                the Cartesian topology as separate local blocks on the
 *                current device ("virtual ranks"; their exchange is a device
 *                copy); the *_ranks entry points then take one field per
 *                rank, and the single-block entry points return
 *                IGG_ERR_STATE.
 *   periods      1 = periodic dimension, 0 = not; NULL = (0,0,0).
 *   overlaps     planes shared by neighbouring local grids, >= 2; NULL=(2,2,2).
 *   me           out, nullable: this process's rank (always 0; virtual ranks
 *                are addressed by index in the *_ranks calls).
 * Pure host work: no HIP call is made.
 * Errors: IGG_ERR_STATE if a grid exists, IGG_ERR_ARG for a bad value. */
int igg_init_global_grid(int nx, int ny, int nz, const int dims[3], const int periods[3],
                         const int overlaps[3], int *me);

/* Global grid size per dimension (Fig. 1 `nx_g()`, `ny_g()`, `nz_g()`):
 * n_g = dims*(n-ol) + ol*(1-period).  Errors: IGG_ERR_STATE, IGG_ERR_ARG. */
int igg_global_size(int64_t n_g[3]);

/* Grid description: any pointer may be NULL.  coords is rank 0's Cartesian
 * position (0,0,0).  Errors: IGG_ERR_STATE. */
int igg_topology(int n[3], int dims[3], int periods[3], int overlaps[3], int coords[3]);

/* Number of ranks the grid holds (the product of dims; Sec. 2 `nprocs`).
 * Errors: IGG_ERR_STATE, IGG_ERR_ARG (null). */
int igg_nranks(int *nranks);

/* Cartesian coordinates of rank `rank` (Sec. 2 `coords`): rank r sits at
 * (r % dims[0], (r / dims[0]) % dims[1], r / (dims[0]*dims[1])), x fastest.
 * Its block holds the points c*(n-ol) + l, l = 0..n-1, of a global index
 * space 0 .. dims*(n-ol)+ol-1 per dimension (one block of that size is the
 * same grid; in a periodic dimension its first and last ol planes are
 * images of each other).
 * Errors: IGG_ERR_STATE, IGG_ERR_ARG (null, rank outside 0..P-1). */
int igg_rank_coords(int rank, int coords[3]);

/* Neighbours of rank `rank` per dimension (Sec. 2 `neighbors`): lower[d] and
 * upper[d] are the ranks one step down and up in dimension d, wrapping in a
 * periodic dimension, -1 at the edge of a non-periodic one (a periodic
 * dimension with dims 1 is its own neighbour).
 * Errors: IGG_ERR_STATE, IGG_ERR_ARG. */
int igg_neighbors(int rank, int lower[3], int upper[3]);

/* Halo update of up to IGG_MAX_FIELDS fields (Fig. 1 `update_halo!`, Sec. 2).
 * For each dimension in the order x, y, z, and each periodic one: pack the
 * planes ol_A-1 and n_A-ol_A of every field into send buffers, exchange them
 * with the neighbours (the lower neighbour receives plane ol_A-1 into its
 * last plane, the upper one plane n_A-ol_A into its first plane; here both
 * neighbours are the process itself), and unpack them into planes n_A-1 and
 * 0.  Full planes move, so edges and corners come out right.
 * With the process as its own neighbour the three phases of a dimension run
 * in one launch, each thread carrying its elements through all three.
 * A field may have the grid size n or n+1 per dimension (staggered faces);
 * its overlap is then ol_A = ol + (n_A - n).  Non-periodic dimensions are
 * left as they are.  Fields may have different element types.
 * Errors: IGG_ERR_STATE, IGG_ERR_ARG (null, nfields outside 1..IGG_MAX_FIELDS,
 * reserved != 0), IGG_ERR_SIZE, IGG_ERR_DTYPE, IGG_ERR_ALIAS (two fields with
 * the same data pointer), IGG_ERR_HIP. */
int igg_update_halo(const igg_field *fields, int nfields, void *stream);

/* igg_update_halo for every rank of the grid: fields[r*nfields + f] is field
 * f of rank r (nfields fields per rank, all of one field index f alike in
 * size and dtype).  Per dimension, in the order x, y, z: each rank packs its
 * planes ol_A-1 and n_A-ol_A into its send buffers, which are copied into
 * the receive buffers of its lower and upper neighbours, and unpacked into
 * their planes n_A-1 and 0; with one rank this is igg_update_halo.
 * Errors: as igg_update_halo; IGG_ERR_SIZE if a field differs in size or
 * dtype from the same field of rank 0. */
int igg_update_halo_ranks(const igg_field *fields, int nfields, void *stream);

/* Finalize the grid (Fig. 1 `finalize_global_grid`): wait for the library's
 * stream, free buffers, stream and events, forget the grid.
 * Errors: IGG_ERR_STATE if no grid exists, IGG_ERR_HIP. */
int igg_finalize_global_grid(void);

/* ---------------------------------------------------------- step (Fig. 1) */

/* One explicit diffusion step fused with the halo update of T2, i.e. the
 * body of Fig. 1's time loop:
 *   T2 = T + dt*(lam*Ci*(d2x(T)/dx^2 + d2y(T)/dy^2 + d2z(T)/dz^2))
 * on the inner points, d2x(T) = (T[i+1]-T[i]) - (T[i]-T[i-1]), followed by
 * igg_update_halo(T2).  T, T2 and Ci must have the grid size n and one
 * element type; T must carry a valid halo (the previous step's update).
 *   split  boundary widths (Fig. 1 `@hide_communication (16, 2, 2)`), counted
 *          from the array edge including the halo plane, each >= overlap.
 *          The boundary slabs the halo update reads are computed first, and
 *          the update of T2 follows them while the inner region is computed.
 *          The x exchange is stored by the step kernels as they compute the
 *          points it moves, so the x slabs are computed with the inner
 *          region.  Schedules (IGG_SCHEDULE):
 *            1  slabs, then the update, on the library's helper stream while
 *               the inner region runs on `stream`, which finally waits for
 *               the helper (the paper's arrangement);
 *            0  slabs first on `stream`, the update on the helper stream;
 *            2  slabs, update and inner region as one chain on `stream`;
 *            3  on one rank that is periodic in every dimension: slabs and
 *               inner region in one launch on `stream`, whose first
 *               work-groups compute the slabs and store the y and z halo
 *               planes of T2 as they go (with IGG_SLAB_PACK=1 they fill send
 *               buffers that one copy then unpacks).
 *          Default: 3 where it applies (measured fastest at 512^3, below the
 *          unsplit step); otherwise 1 for inner regions of 2^21 points and
 *          more in FP64/FP32, 2 for smaller ones and for FP16.
 *          NULL = no overlap: the whole step, then the halo update, on
 *          `stream`.
 *   rnd    FP16 store rounding, NULL = round to nearest even (ignored for
 *          FP64/FP32).
 * Arithmetic: FP64 for IGG_F64; FP32 for IGG_F32 and IGG_F16 with dt*lam and
 * 1/dd^2 rounded once from FP64.  The result does not depend on `split`.
 * Errors: IGG_ERR_STATE, IGG_ERR_ARG, IGG_ERR_SIZE, IGG_ERR_DTYPE,
 * IGG_ERR_ALIAS (T2 overlapping T or Ci), IGG_ERR_HIP. */
int diffusion_step(const igg_field *T2, const igg_field *T, const igg_field *Ci, double lam,
                   double dt, double dx, double dy, double dz, const int split[3],
                   const igg_rounding *rnd, void *stream);

/* diffusion_step for every rank of the grid: T2[r], T[r] and Ci[r] are rank
 * r's blocks (arrays of nranks fields, no block sharing memory with
 * another).  The step runs on each block, the x exchange stores into the x
 * neighbours' blocks, and one igg_update_halo_ranks of T2 follows, with the
 * same split schedule as diffusion_step.  FP16 stochastic rounding hashes
 * each point's global index, so the result equals the single-block run of
 * the global grid bit for bit.
 * Errors: as diffusion_step, naming the rank. */
int diffusion_step_ranks(const igg_field *T2, const igg_field *T, const igg_field *Ci, double lam,
                         double dt, double dx, double dy, double dz, const int split[3],
                         const igg_rounding *rnd, void *stream);

/* nt steps of Fig. 1's time loop on the buffers T and T2, which swap every
 * step (step it reads buf[it % 2] and writes the other, buf = {T, T2}), with
 * the same arguments as diffusion_step; *final_buf is set to the index of
 * the buffer holding T_nt (0: T, 1: T2).  T2 must hold T's halo planes in
 * non-periodic dimensions (Fig. 1 starts it as a copy of T).  rnd: the
 * stochastic-rounding counter advances by one per step.
 *   use_graph  0: every step is launched as diffusion_step would.  1: up to
 *          8 pairs of steps T -> T2 -> T are captured once into a HIP graph
 *          on a library stream and replayed on `stream`; the steps left over
 *          run directly.  The graph is kept for later calls with identical
 *          arguments (and pair count) and rebuilt when any differs.  For
 *          grids small enough that launch latency dominates.  Stochastic
 *          rounding needs a new counter every step, so it refuses
 *          use_graph = 1.
 * Results are bit-identical for both values of use_graph.
 * Errors: as diffusion_step; IGG_ERR_ARG for nt < 0, a null final_buf, or
 * use_graph with stochastic rounding. */
int diffusion_run(const igg_field *T, const igg_field *T2, const igg_field *Ci, double lam, double dt,
                  double dx, double dy, double dz, const int split[3], const igg_rounding *rnd, int nt,
                  int use_graph, int *final_buf, void *stream);

/* Stable time step of Fig. 1: dt = min(dx^2,dy^2,dz^2)/lam/maximum(Ci)/6.1,
 * the maximum taken in FP64 over every point of Ci on the GPU.
 * Synchronises `stream`.  Errors: as igg_reduce, IGG_ERR_ARG for lam <= 0. */
int diffusion_dt(const igg_field *Ci, double lam, double dx, double dy, double dz, double *dt,
                 void *stream);

/* Adjoint of diffusion_step.  With a = dt*lam and L the operator
 * sum_d d2_d(.)/dd^2, the step is T_{n+1} = T_n + a*Ci.*(L T_n); given the
 * incoming adjoint lam_np1 = dLoss/dT_{n+1} (with a valid halo) it computes
 *   lam_n = lam_np1 + a*L(Ci.*lam_np1)     (inner points), then halo(lam_n)
 *   gCi  += a*lam_np1.*(L T_n)             (inner points; halo untouched)
 * T_n is the state the forward step read (valid halo); Ci needs a valid halo.
 * lam_np1 lives on the unique points: its halo is their periodic image in
 * periodic dimensions and zero in non-periodic ones (lam_n's halo planes in
 * non-periodic dimensions are not written, so start lam_n zeroed there).
 * FP64 or FP32 (IGG_ERR_DTYPE for FP16).  `split` as in diffusion_step,
 * except that by default the slabs, the update and the inner region run as
 * one chain on `stream` at every size (the adjoint kernel is partly
 * latency-bound and runs slower with the slabs beside it); on one rank that
 * is periodic in every dimension, one launch computes every inner point and
 * stores lam_n's halo with it (the x exchange, and each y/z halo point from
 * the inner point that is its image).
 * Errors: as diffusion_step; IGG_ERR_ALIAS if lam_n or gCi overlaps an input
 * or each other. */
int diffusion_step_adjoint(const igg_field *lam_n, const igg_field *lam_np1,
                           const igg_field *T_n, const igg_field *Ci, const igg_field *gCi,
                           double lam, double dt, double dx, double dy, double dz,
                           const int split[3], void *stream);

/* diffusion_step_adjoint for every rank of the grid: each argument is an
 * array of nranks fields, rank r's blocks (no output block sharing memory
 * with another block).  The x exchange of lam_n stores into the x
 * neighbours' blocks and one igg_update_halo_ranks of lam_n follows, so the
 * result equals the adjoint step on one block of the global grid bit for
 * bit.  Errors: as diffusion_step_adjoint, naming the rank. */
int diffusion_step_adjoint_ranks(const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                                 const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx,
                                 double dy, double dz, const int split[3], void *stream);

/* ---------------------------------------------- staggered flux form */

/* Flux form of the same step on the staggered grid (Sec. 2 "regular
 * staggered grid"): face fluxes qx (nx+1,ny,nz), qy (nx,ny+1,nz),
 * qz (nx,ny,nz+1) with face f between cells f-1 and f,
 *   qx[f] = -lam*(T[f]-T[f-1])/dx       faces 1..nx-1 of the inner rows
 *   T2    = T - dt*Ci*((qx[i+1]-qx[i])/dx + (qy[j+1]-qy[j])/dy + (qz[k+1]-qz[k])/dz)
 * then one halo update of {T2, qx, qy, qz}.  FP64 or FP32.  One pass per
 * cell computes its lower faces (and the upper face of the last cell of a
 * row, column or plane), the update from its six faces, and, for periodic
 * x, the x exchange of all four fields; the values equal a face pass
 * followed by a cell pass.
 *   split  boundary widths as in diffusion_step, each >= overlap + 1 (the
 *          face fields overlap by one more plane in their own dimension);
 *          the y and z slabs are computed first, the halo update of the four
 *          fields follows them on the helper stream beside the inner
 *          region.  NULL = no overlap.
 * Errors: as diffusion_step (IGG_ERR_ARG for a split width below ol+1). */
int diffusion_flux_step(const igg_field *T2, const igg_field *T, const igg_field *Ci,
                        const igg_field *qx, const igg_field *qy, const igg_field *qz, double lam,
                        double dt, double dx, double dy, double dz, const int split[3], void *stream);

/* diffusion_flux_step for every rank of the grid: each argument is an array
 * of nranks fields (rank r's blocks; the face fields one point longer in
 * their own dimension).  The x exchange of all four fields stores into the
 * x neighbours' blocks and one igg_update_halo_ranks of {T2, qx, qy, qz}
 * follows; the result equals the flux step on one block of the global grid
 * bit for bit.  Errors: as diffusion_flux_step, naming the rank. */
int diffusion_flux_step_ranks(const igg_field *T2, const igg_field *T, const igg_field *Ci,
                              const igg_field *qx, const igg_field *qy, const igg_field *qz, double lam,
                              double dt, double dx, double dy, double dz, const int split[3], void *stream);

/* Adjoint of diffusion_flux_step.  With mu = Ci.*lam_np1 and the face
 * fluxes p = -lam*grad(mu) and q_n = -lam*grad(T_n) (the forward fluxes of
 * step n) formed per cell from its neighbours, as the forward pass forms q:
 *   lam_n = lam_np1 - dt*div(p)              (inner cells), then halo(lam_n)
 *   gCi  += -dt*lam_np1.*div(q_n)            (inner cells; halo untouched)
 * T_n is the state the forward step read (valid halo); Ci needs a valid
 * halo.  FP64 or FP32.  `split` as in diffusion_step_adjoint (widths >=
 * overlap).
 * Errors: as diffusion_step_adjoint. */
int diffusion_flux_step_adjoint(const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                                const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx,
                                double dy, double dz, const int split[3], void *stream);

/* diffusion_flux_step_adjoint for every rank of the grid (arrays of nranks
 * fields, as diffusion_step_adjoint_ranks).  Errors: as
 * diffusion_flux_step_adjoint, naming the rank. */
int diffusion_flux_step_adjoint_ranks(const igg_field *lam_n, const igg_field *lam_np1, const igg_field *T_n,
                                      const igg_field *Ci, const igg_field *gCi, double lam, double dt, double dx,
                                      double dy, double dz, const int split[3], void *stream);

/* --------------------------------------------------------- reductions */

/* FP64 reduction of one or two fields (IGG_RED_*); b is needed by
 * SUM_RATIO, HALF_SQDIFF, DOT and MAX_ABS_DIFF and ignored otherwise.  Any
 * element type; values are widened to FP64 before they are combined, in a
 * fixed order, so repeated calls give identical bits.  The result is written
 * to *out (host memory) after `stream` is synchronised.
 * Errors: IGG_ERR_STATE, IGG_ERR_ARG, IGG_ERR_SIZE (a, b differ),
 * IGG_ERR_DTYPE, IGG_ERR_HIP. */
int igg_reduce(int op, const igg_field *a, const igg_field *b, double *out, void *stream);

/* Seed of the adjoint sweep and restriction of a gradient to the unique
 * points (the loss 0.5*||T_nt - T_obs||^2 over the inner points and its
 * gradient lam = T_nt - T_obs, which lives on the inner points):
 *   lam = T - T_obs on the inner points (T alone when T_obs is NULL, zero
 *         when T is NULL too), zero on every halo point; then, with halo = 1,
 *         the halo update of lam (periodic images; non-periodic halo planes
 *         stay zero), as diffusion_step_adjoint expects of its input.
 *   loss  nullable; needs T_obs: the FP64 loss, with the bits of igg_reduce
 *         IGG_RED_HALF_SQDIFF on (T, T_obs); synchronises `stream`.
 * T, T_obs and lam have the grid size and one element type (caller-owned);
 * lam may not overlap T or T_obs.  One pass over the fields (and, with
 * halo = 1, the halo launches).
 * On a grid of virtual ranks each block is seeded alone (halo = 0) and one
 * igg_update_halo_ranks follows.
 * Errors: IGG_ERR_STATE (halo = 1 on a grid of virtual ranks), IGG_ERR_ARG
 * (T_obs without T, loss without T_obs, halo not 0/1), IGG_ERR_SIZE,
 * IGG_ERR_DTYPE, IGG_ERR_ALIAS, IGG_ERR_HIP. */
int igg_adjoint_seed(const igg_field *T, const igg_field *T_obs, const igg_field *lam, int halo, double *loss,
                     void *stream);

/* igg_reduce for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same reduction over the same points with the same kernels, so the same
 * bits as igg_reduce, but:
 *   out_dev  device pointer to one double (caller-owned), written on
 *            `stream`; the call does not synchronise and returns once the
 *            work is queued.
 *   - No allocation of any kind: the partial results go to a static device
 *     array of 1024 doubles (8 KiB per device, held until the process
 *     ends), which bounds the work-groups of one reduction at 1024 (every
 *     reduction fits; IGG_ERR_SIZE otherwise); the grid's own buffers and
 *     streams are neither made nor used (only igg_init_global_grid is
 *     needed, for the size checks).
 *   - Every call on a device shares that array: calls that overlap in time
 *     on one device (unordered streams, several host threads) race.
 * Errors: as igg_reduce (IGG_ERR_ARG for a null out_dev). */
int igg_reduce_noalloc(int op, const igg_field *a, const igg_field *b, double *out_dev, void *stream);

/* --------------------------------------------------------- host helpers */

/* The boundary-first partition used by diffusion_step for grid size n and
 * widths split: up to 6 disjoint boundary boxes followed by the inner box,
 * each as {i0,i1,j0,j1,k0,k1} (half-open).  Empty boxes are dropped; the
 * inner box is last and may be empty (i0 == i1).  *nboxes counts all boxes
 * written.  Pure host function.  Errors: IGG_ERR_ARG. */
int igg_plan_split(const int n[3], const int split[3], int boxes[7][6], int *nboxes);

/* Kernel timing.  While enabled, each launch of the inner-region kernel of
 * diffusion_step / diffusion_step_adjoint (and the fused pass of
 * diffusion_flux_step) is bracketed by two HIP events on the stream it runs
 * on, and so are the boundary-slab kernels of a split step.  The events
 * carry no system-scope fence; enabling creates a pool of them for 1024
 * launches on the current device, so timed work does not pay for their
 * creation.
 * igg_timing_read synchronises those events and returns the summed
 * inner-kernel duration in milliseconds, its launch count, the inner points
 * those launches computed, and the summed boundary-kernel duration (any
 * pointer may be NULL), then resets the totals.  Errors: IGG_ERR_STATE,
 * IGG_ERR_HIP (enabling makes the event pool, so it needs the GPU). */
int igg_timing_enable(int on);
int igg_timing_read(double *ms, int64_t *launches, int64_t *points, double *boundary_ms);

/* Streaming-bandwidth probe: the HBM rate a plain stream of a given
 * read/write mix reaches on the current device, the achievable ceiling the
 * stencil kernels are compared with beside the vendor peak.  For i < n:
 * dst[w][i] = src[0][i] + ... + src[nsrc-1][i] (FP64) for every w, each
 * array read or written once, with 16-byte non-temporal accesses, one
 * vector per array and thread in work-groups of 256 threads.
 *   src, dst   host arrays of nsrc (1..4) and ndst (1..4) device pointers to
 *              n doubles each, 16-byte aligned; the caller owns them.
 *   n          doubles per array, even.
 * Needs no grid.  Asynchronous on `stream`.
 * Errors: IGG_ERR_ARG (null or misaligned pointer, counts out of range),
 * IGG_ERR_HIP. */
int igg_stream_probe(const void *const *src, int nsrc, void *const *dst, int ndst, int64_t n, void *stream);

/* Message for the calling thread's last failure ("" if none). */
const char *igg_last_error(void);

/* Library version string. */
const char *igg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IGG_MI355X_H */
