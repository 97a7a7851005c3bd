/*
 * fga.h -- C ABI of the MI355X (gfx950) frozen Gaussian approximation path.
 *
 * The library computes the paper's three-step algorithm (Yang, Lu and Fomel,
 * "Seismic modeling using the frozen Gaussian approximation", Algorithm
 * section) for the 2-D acoustic wave equation u_tt = c(x)^2 Lap u:
 *
 *   fga_decompose    step 1: FBI transform of f0 (and f1) on a (q,p) mesh
 *                    (psi eq. and the local fast FBI of the Initial wavefield
 *                    decomposition section), branch data u_{+-,0}, relative
 *                    thresholding, initial beam state;
 *   fga_propagate    step 2: RK4 of the ray equations (characline eq.) for
 *                    H = +-c(Q)|P| (hamiltonian eq.), the dynamic ray tracing
 *                    equations (dzQ, dzP eqs.) and the amplitude equation
 *                    (a_formu eq.);
 *   fga_reconstruct  step 3: the frozen-Gaussian sum (recons eq.) on the grid;
 *   fga_trace        step 3 at receiver nodes at every rec_every-th step;
 *   fga_trace_adjoint, fga_decompose_adjoint
 *                    the gradient of a receiver misfit with respect to the
 *                    velocity samples and the initial wavefield;
 *   fga_reconstruct_adjoint, fga_propagate_ckpt, fga_propagate_adjoint
 *                    the same for a misfit of the whole field u(T): the
 *                    transposes of step 3 and step 2, chained with
 *                    fga_decompose_adjoint.
 *
 * Conventions shared by every entry point
 *   - All pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *     tensors) owned by the caller.  The library owns the context and its
 *     workspaces only.
 *   - All work is enqueued on the context's stream and is asynchronous.
 *     The calls that wait for the stream are: fga_sync_status,
 *     fga_copy_offsets, fga_autotune and fga_graph_capture (always); the
 *     gradient calls with logged dJ/dc (grad_log >= 0 or deterministic = 1,
 *     once per call, to size the reduction); and any call that must grow a
 *     workspace the context owns (it waits before freeing the smaller
 *     buffer, which happens on the first call of a new size or mode, so a
 *     repeated call of the same shape does not wait).  Growing a workspace
 *     makes a captured graph stale (see fga_graph_launch).
 *   - Grid arrays are C-ordered [n2][n1] float64 on nodes x_i = o + i*d
 *     (axis 1 horizontal and fastest, axis 2 depth).
 *   - Errors in arguments return immediately with FGA_EINVAL and leave the
 *     stream untouched.  Errors found on the device (capacity overflow,
 *     non-finite values, c <= 0) set a sticky status word that
 *     fga_sync_status reads.  fga_last_error() describes the last failure.
 */
#ifndef FGA_H
#define FGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fga_ctx fga_ctx;

typedef enum {
    FGA_OK = 0,
    FGA_EINVAL = -1,     /* invalid argument (checked on the host)          */
    FGA_ENOMEM = -2,     /* device allocation of a workspace failed         */
    FGA_ECAPACITY = -3,  /* more beams kept than the beam buffer holds      */
    FGA_EHIP = -4,       /* a HIP runtime call failed                       */
    FGA_ENUMERIC = -5,   /* NaN/Inf in an input or a beam state, or c <= 0  */
    FGA_ESTATE = -6      /* call out of order (e.g. no velocity set)        */
} fga_status;

typedef enum {
    FGA_FP64 = 0,   /* every stage in double precision                       */
    FGA_MIXED = 1,  /* FP32 FBI and splat (phase reduced mod 2 pi in FP64),
                       FP64 ray/amplitude integration                        */
    FGA_MIXED_SPLIT = 2  /* as FGA_MIXED, with the FP32 products of FBI
                       pass 2 and of the splat formed on the FP16 matrix
                       cores from hi/lo splits of both operands
                       (x = fp16(x) + fp16(x - fp16(x)), about 2^-22
                       relative; the pass-1 output and the splat's U scaled
                       per shot by a power of two to stay in the FP16 range)
                       and accumulated in FP32 (then FP64 in the splat).
                       The splat's box decides which 64 x 64 tiles a beam
                       visits; inside them its Gaussian is not cut at the
                       box (the terms beyond it are below tau_win).
                       Beyond 8192 (shot, tile) pairs the splat keeps the
                       FP32 products.                                        */
} fga_precision;

/* Node-centred grid: x1 = o1 + i1*d1 (i1 < n1), x2 = o2 + i2*d2 (i2 < n2),
 * 4 <= n1, n2 <= FGA_MAX_N (truncation boxes keep node indices in 16 bits). */
#define FGA_MAX_N 32767
typedef struct {
    int32_t n1, n2;
    double o1, o2, d1, d2;
} fga_grid;

/* Numerical parameters (lengths in the grid's units).
 *   eps        the high-frequency parameter (rescaled wavelength)
 *   q-mesh     grid nodes (qb1 + j1*qs1, qb2 + j2*qs2), j1 < nq1, j2 < nq2
 *   p-mesh     p_l = (l - (np-1)/2) * dp per axis; np1, np2 even, so p = 0
 *              is never a node
 *   tau        keep (branch, q, p) with |psi| >= tau * max|psi| (per shot,
 *              over both branches) and |psi| > 0 (thresholding paragraph of
 *              the Initial wavefield decomposition section); used when
 *              top_n = 0
 *   top_n      if > 0: each branch of each shot keeps instead its top_n
 *              largest |psi| (the N-largest selection of the Numerical test
 *              section), equal magnitudes in increasing candidate order,
 *              never |psi| = 0 (so fewer when fewer are nonzero).  The
 *              magnitudes are compared in the precision of the FBI (FP32 in
 *              FGA_MIXED)
 *   amp_closed 0: integrate the amplitude equation (a_formu eq.); 1: set
 *              a = c(Q)/c(q) (det Z)^{1/2} after every step instead (the
 *              closed form the Formulation section derives from the
 *              conserved a^2/(c(Q)^2 det Z)), the square root taken nearest
 *              the previous step's so that it is continuous in time.  The
 *              gradient entry points require 0.
 *   dz_divided 0: integrate the dynamic ray tracing equations (dzQ, dzP
 *              eqs.) for A = dzQ, B = dzP; 1: take them by divided
 *              differences instead (the alternative named next to those
 *              equations): every beam also advances, by the same RK4, the
 *              eight rays started at (q +- h_j e_j, p) and (q, p +- h_{2+j}
 *              e_j), h = dz_scale (qs1 d1, qs2 d2, dp1, dp2), and after
 *              every step
 *              dq_j Q_k = (Q_k(+q_j) - Q_k(-q_j)) / (2 h_j),
 *              dp_j Q_k likewise over 2 h_{2+j} (and P alike),
 *              A[j][k] = dq_j Q_k - i dp_j Q_k, B[j][k] = dq_j P_k - i dp_j P_k.
 *              The extra rays start from the incoming state along its A and
 *              B (exactly the displaced nodes' rays at t = 0), so a run in
 *              segments restarts them from the stored A, B.  Requires
 *              amp_closed = 1 (the amplitude follows from det Z).
 *   dz_scale   spacing of the divided differences in mesh steps (> 0;
 *              read when dz_divided = 1): 1 takes the neighbouring mesh
 *              nodes; smaller values take rays closer than the mesh, which
 *              approach the dynamic ray tracing values at second order
 *   deterministic  0: the gradient entry points add dJ/dc with FP64 atomics
 *              (rounding order not fixed); 1: every beam logs its dJ/dc
 *              contributions in its own slots and the logs are reduced in a
 *              fixed order (stable sort by knot cell, then by beam and
 *              sequence; every knot sums its cells in a fixed order), so
 *              repeated calls give bit-identical dc.  The gradient calls then
 *              synchronise the stream once to size the reduction.
 *   grad_log   (deterministic = 0) where the gradient kernels put dJ/dc
 *              (a record = the 16 knot sums of one B-spline cell):
 *              0 (automatic): each beam logs its records in its own slots,
 *              up to min(4 steps + 1, what fits the smaller of
 *              FGA_GRAD_LOG_BYTES and half the free device memory for the
 *              beam capacity) of them; the logs are then summed by cell in a
 *              fixed order (the deterministic mode's reduction, which
 *              synchronises the stream once per call to size its sort);
 *              records past a beam's slots are added with FP64 atomics where
 *              they are made.  n > 0: at most n slots per beam (no size
 *              cap).  -1: no logs, every record is added with atomics where
 *              it is made, and the call does not synchronise (also what a
 *              call does when the logs cannot be allocated).  The three give
 *              the same dc up to the rounding order.  The logged form is the
 *              faster one here: atomics from many rays into the same cells
 *              contend, and the integrating waves wait on them.
 *   ckpt_every_step  0: fga_trace and fga_propagate_ckpt store the state
 *              at the start of every record segment, and the adjoints
 *              recompute each segment from it; 1: they store the state
 *              before every RK4 step and the final state,
 *              ckpt_dev[nsteps + 1][FGA_NSTATE][capacity] with nsteps =
 *              nrec_t * rec_every (nseg * seg), and the adjoints read those
 *              states instead of recomputing them (23 doubles per beam and
 *              step of memory for about a fifth of the adjoint's
 *              arithmetic).  Requires amp_closed = 0 and dz_divided = 0.
 *   tau_fbi    the FBI box B_eps has half-width ceil(sqrt(2 eps ln(1/tau_fbi))/d)
 *   tau_win    each Gaussian is summed over the box of half-width
 *              ceil(sqrt(2 eps ln(1/tau_win))/d) around the node nearest Q
 *   dt         RK4 time step                                                */
typedef struct {
    double eps;
    int32_t qb1, qb2, qs1, qs2, nq1, nq2;
    int32_t np1, np2;
    double dp1, dp2;
    double tau, tau_fbi, tau_win;
    double dt;
    int32_t top_n;
    int32_t amp_closed;
    int32_t dz_divided;
    double dz_scale;
    int32_t deterministic;
    int32_t grad_log;
    int32_t ckpt_every_step;
} fga_params;

/* Size cap of the automatic dJ/dc logs of one context (grad_log = 0); a
 * call also keeps them within half of the free device memory.             */
#define FGA_GRAD_LOG_BYTES (96LL << 30)

/* Beam storage: structure of arrays in one float64 buffer
 * f[FGA_NFIELD][capacity] (field-major), caller-allocated on the device.
 *   field 0..3   q1, q2, p1, p2          the (q,p) mesh node of the beam
 *   field 4..5   C = w psi / (2 pi eps)^3 (re, im), w = qs1 d1 qs2 d2 dp1 dp2
 *   field 6..28  state: Q1, Q2, P1, P2, S, A = dzQ (2x2 complex, row-major,
 *                re/im interleaved), B = dzP (same), a (re, im)
 * id[capacity] (int64) is the candidate index
 *   ((shot*2 + (branch == -1)) * nq1*nq2 + j2*nq1 + j1) * np1*np2 + l2*np1 + l1,
 * from which shot, branch, q and p follow.  Beams are stored in increasing
 * id.  offsets[nshots+1] (int64, device) delimit the beams of each shot. */
#define FGA_NSTATE 23
#define FGA_NFIELD 29
#define FGA_F_STATE 6

typedef struct {
    int64_t capacity;
    double *f;
    int64_t *id;
    int64_t *offsets;
} fga_beams;

/* Create a context for one grid, one parameter set and one precision.
 * max_shots bounds nshots of later calls (workspaces are sized for it).
 * stream is a hipStream_t (NULL = the default stream).                     */
fga_status fga_create(fga_ctx **ctx, const fga_grid *grid, const fga_params *params,
                      int32_t precision, int32_t max_shots, void *stream);
fga_status fga_destroy(fga_ctx *ctx);
fga_status fga_set_stream(fga_ctx *ctx, void *stream);

/* Copy the velocity c[n2][n1] (device, float64, c > 0) into the context.
 * c(x) between nodes is the uniform cubic B-spline with these samples as
 * coefficients, indices clamped to the grid.                               */
fga_status fga_set_velocity(fga_ctx *ctx, const double *c_dev);

/* Step 1 for nshots shots: f0_dev, f1_dev are [nshots][n2][n1] (f1_dev may
 * be NULL for f1 = 0).  Writes beams->f, beams->id and beams->offsets.
 * If more than beams->capacity beams are kept, the first capacity beams (in
 * id order) are written, offsets are clipped, and the status word reports
 * FGA_ECAPACITY with the number needed.                                    */
fga_status fga_decompose(fga_ctx *ctx, int32_t nshots, const double *f0_dev,
                         const double *f1_dev, fga_beams *beams);

/* Step 2: advance every beam by nsteps RK4 steps of size params.dt.        */
fga_status fga_propagate(fga_ctx *ctx, fga_beams *beams, int32_t nshots, int32_t nsteps);

/* Step 3: u_dev[nshots][n2][n1] = Re sum over each shot's beams.  u_dev is
 * overwritten.                                                             */
fga_status fga_reconstruct(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                           double *u_dev);

/* Receiver traces: nrec_t times, advance rec_every steps then evaluate the
 * sum at the nrec nodes rec_dev[] (flat i2*n1 + i1, int32, device).
 * traces_dev[nshots][nrec_t][nrec].  The beams end at t = nrec_t*rec_every*dt.
 * If ckpt_dev is not NULL it receives the beam states before every segment:
 * ckpt_dev[k][FGA_NSTATE][capacity], k < nrec_t (with ckpt_every_step = 1:
 * before every step and at the end, [nrec_t * rec_every + 1][...]).       */
fga_status fga_trace(fga_ctx *ctx, fga_beams *beams, int32_t nshots,
                     const int32_t *rec_dev, int32_t nrec, int32_t rec_every,
                     int32_t nrec_t, double *traces_dev, double *ckpt_dev);

/* fga_trace for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments and results, but the receiver classification and the
 * partial receiver sums live in a static device array of
 * FGA_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends (its address is looked up once per device by fga_create), so
 * the call allocates and frees nothing.  The partial sums need
 * nshots * nrec * 8 bytes per work split: when the default split count does
 * not fit, fewer splits are used (the traces then agree with fga_trace's to
 * the rounding of the sum order); if even one split does not fit
 * (nshots * nrec * 8 + 256 > FGA_NOALLOC_SCRATCH_BYTES) the call returns
 * FGA_EINVAL before any launch.  All calls on one GPU share the array: two
 * such calls that overlap in time on that GPU (other streams, other
 * contexts, other threads) race and give wrong traces; calls ordered on one
 * stream are safe.  FGA_ESTATE if the context has no scratch address (more
 * than 64 devices).                                                        */
#define FGA_NOALLOC_SCRATCH_BYTES (16LL << 20)
fga_status fga_trace_noalloc(fga_ctx *ctx, fga_beams *beams, int32_t nshots,
                             const int32_t *rec_dev, int32_t nrec, int32_t rec_every,
                             int32_t nrec_t, double *traces_dev, double *ckpt_dev);

/* Adjoint of fga_trace: the gradient of J = 1/2 sum (traces - data)^2
 * through the RK4 integration of the ray, dynamic ray tracing and amplitude
 * equations and the receiver sums, with the beam set and every truncation
 * box held fixed (the exact gradient of the discrete forward).
 *   beams      the beams of the forward call (their coefficients C and ids
 *              are read; the states are not)
 *   rec, nrec, rec_every, nrec_t   as in the forward fga_trace call
 *   ckpt_dev   the checkpoints that fga_trace wrote ([nrec_t][23][capacity],
 *              or every step's with ckpt_every_step = 1)
 *   gtr_dev    dJ/dtraces [nshots][nrec_t][nrec] (e.g. traces - data)
 *   dc_dev     [n2][n1]: dJ/dc is ADDED (caller zeroes it first), in the
 *              order that deterministic and grad_log describe
 *   gcoef_dev  [2][capacity]: dJ/d(Re C, Im C) per beam, overwritten
 * Scratch of rec_every * 23 doubles per beam capacity is held by the
 * context (none with ckpt_every_step = 1).                                 */
fga_status fga_trace_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                             const int32_t *rec_dev, int32_t nrec, int32_t rec_every,
                             int32_t nrec_t, const double *ckpt_dev, const double *gtr_dev,
                             double *dc_dev, double *gcoef_dev);

/* Adjoint of fga_reconstruct for a misfit J(u) of the field: from
 * du_dev = dJ/du [nshots][n2][n1] to the cotangents of every beam's current
 * state and coefficient, through the recons eq. with every truncation box
 * held fixed (FP64 in both precision modes; the boxes are those of the
 * context's tau_win, as in the forward call).
 *   dstate_dev [FGA_NSTATE][capacity], overwritten for the beams in offsets:
 *              dJ/dQ1, dQ2, dP1, dP2, dS, zeros for dzQ and dzP (u does not
 *              read them), dJ/d(Re a), dJ/d(Im a)
 *   dcoef_dev  [2][capacity]: dJ/d(Re C, Im C), overwritten
 * The beams are read, not changed.                                         */
fga_status fga_reconstruct_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                   const double *du_dev, double *dstate_dev, double *dcoef_dev);

/* Propagation that keeps checkpoints for fga_propagate_adjoint: nseg
 * segments of seg RK4 steps each (as nseg calls of fga_propagate), the state
 * at the start of segment k written to ckpt_dev[k][FGA_NSTATE][capacity]
 * (with ckpt_every_step = 1 every step's and the final state,
 * [nseg * seg + 1][FGA_NSTATE][capacity]).                                 */
fga_status fga_propagate_ckpt(fga_ctx *ctx, fga_beams *beams, int32_t nshots, int32_t seg,
                              int32_t nseg, double *ckpt_dev);

/* Adjoint of fga_propagate_ckpt: the cotangent of the state after the
 * nseg*seg steps (dstate_dev [FGA_NSTATE][capacity] on entry, e.g. from
 * fga_reconstruct_adjoint) is pulled back through the RK4 of the ray,
 * dynamic ray tracing and amplitude equations to the cotangent of the state
 * before them (dstate_dev on return); dJ/dc through the velocity in every
 * step is ADDED to dc_dev [n2][n1] (in the order that deterministic and
 * grad_log describe).  ckpt_dev as written by the forward call.  Requires
 * amp_closed = 0 (hence dz_divided = 0).  Scratch of seg * 23 doubles per
 * beam capacity is held by the context (none with ckpt_every_step = 1).    */
fga_status fga_propagate_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                 int32_t seg, int32_t nseg, const double *ckpt_dev,
                                 double *dstate_dev, double *dc_dev);

/* Adjoint of fga_decompose for the beams it kept (the threshold set is held
 * fixed): from dJ/dC (gcoef_dev, [2][capacity]) to dJ/df0 (df0_dev
 * [nshots][n2][n1], overwritten) through C = w psi_{+-}/(2 pi eps)^3,
 * u_{+-,0} (psi eq.) and the transposed windowed DFTs.  When the forward
 * call had f1 != NULL, df1_dev receives dJ/df1 and dJ/dc through c(q) is
 * ADDED to dc_dev (both then required).  Uses the FBI output of the most
 * recent fga_decompose on this context, which must have produced beams.    */
fga_status fga_decompose_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                 const double *gcoef_dev, double *df0_dev, double *df1_dev,
                                 double *dc_dev);

/* Batched forward under a HIP graph (many shots with uneven beam counts in
 * one set of launches: every kernel reads the per-shot beam ranges from the
 * device offsets, so nothing is read back on the host).  fga_graph_capture
 * runs decompose -> propagate(nsteps) -> reconstruct once on the context's
 * stream (sizing every workspace), then records the same sequence into a
 * graph on a context-owned capture stream and instantiates it; the stream
 * must not be capturing already.  fga_graph_launch replays it on the
 * context's stream with the pointers given at capture (update the inputs in
 * place between replays).  A later capture replaces the graph.  A call on
 * this context that reallocates one of its workspaces after the capture (a
 * larger beam capacity or shot count, fga_autotune trying a larger split,
 * the gradient calls' buffers) frees memory the graph addresses: from then
 * on fga_graph_launch returns FGA_ESTATE without launching, until the next
 * fga_graph_capture.                                                       */
fga_status fga_graph_capture(fga_ctx *ctx, int32_t nshots, const double *f0_dev,
                             const double *f1_dev, fga_beams *beams, int32_t nsteps,
                             double *u_dev);
fga_status fga_graph_launch(fga_ctx *ctx);

/* Splat autotuner: times fga_reconstruct of these (already propagated)
 * beams for a ladder of work splits (wavefronts per CU for the mixed MFMA
 * splat, workgroups per CU for the FP64 splat), keeps the fastest for this
 * context and appends it to the JSON-lines cache cache_path (may be NULL),
 * keyed by grid size, window, precision, shot count and CU count; a cached
 * key is reused without timing.  u_dev is overwritten.  *chosen (may be
 * NULL) receives the choice.  Synchronises the stream.                     */
fga_status fga_autotune(fga_ctx *ctx, const fga_beams *beams, int32_t nshots, double *u_dev,
                        const char *cache_path, int32_t *chosen);

/* Synchronise the stream, read the sticky device status word and clear it.
 * *needed (may be NULL) receives the beam count a capacity overflow needed. */
fga_status fga_sync_status(fga_ctx *ctx, int64_t *needed);

/* Synchronous copy of beams->offsets[0..nshots] to host memory.            */
fga_status fga_copy_offsets(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                            int64_t *offsets_host);

/* Human-readable description of the last error on this context (or of the
 * last fga_create failure when ctx is NULL).                               */
const char *fga_last_error(const fga_ctx *ctx);

/* ---------------------------------------------------------------------
 * Three space dimensions (FP64): the same three steps for the 3-D acoustic
 * wave equation (the paper states the method for general d; d = 3 here).
 * Grid arrays are C-ordered [n3][n2][n1] float64 on x = o + i*d per axis.
 * Beams use fga_beams with f[FGA3_NFIELD][capacity]:
 *   field 0..2   q1, q2, q3        field 3..5   p1, p2, p3
 *   field 6..7   C = w psi / (2 pi eps)^{9/2} (re, im),
 *                w = prod_a (qs_a d_a) prod_a dp_a
 *   field 8..52  state: Q(3), P(3), S, A = dzQ (3x3 complex, row-major,
 *                re/im interleaved), B = dzP (same), a (re, im);
 *                at t = 0: Q = q, P = p, S = 0, A = I, B = -iI, a = 2^{3/2}
 * id = ((shot*2 + (branch == -1)) * NQ + qflat) * NP + pflat with
 * qflat = (j3*nq2 + j2)*nq1 + j1, pflat = (l3*np2 + l2)*np1 + l1; beams in
 * increasing id; offsets[nshots+1] as in 2-D.  The p-mesh per axis is
 * p_l = (l - (np-1)/2) dp (np even); thresholding, truncation boxes and
 * their half-widths follow the 2-D rules per axis.  Errors as in 2-D; the
 * device status is read by fga3_sync_status.                            */
typedef struct fga3_ctx fga3_ctx;

typedef struct {
    int32_t n1, n2, n3;
    double o1, o2, o3, d1, d2, d3;
} fga3_grid;

typedef struct {
    double eps;
    int32_t qb[3], qs[3], nq[3];   /* q-mesh nodes qb + j*qs per axis   */
    int32_t np[3];
    double dp[3];
    double tau, tau_fbi, tau_win;
    double dt;
} fga3_params;

#define FGA3_NSTATE 45
#define FGA3_NFIELD 53
#define FGA3_F_STATE 8

/* Context for one 3-D grid and parameter set; max_shots bounds nshots.     */
fga_status fga3_create(fga3_ctx **ctx, const fga3_grid *grid, const fga3_params *params,
                       int32_t max_shots, void *stream);
fga_status fga3_destroy(fga3_ctx *ctx);
/* c[n3][n2][n1] (device, c > 0): the tricubic B-spline with these samples
 * as coefficients, indices clamped to the grid.                            */
fga_status fga3_set_velocity(fga3_ctx *ctx, const double *c_dev);
/* Step 1 for nshots shots: f0_dev, f1_dev [nshots][n3][n2][n1] (f1 may be
 * NULL): FBI (psi eq., three separable windowed DFTs over the box),
 * u_{+-,0}, |psi| >= tau max|psi| per shot, beams written in id order.     */
fga_status fga3_decompose(fga3_ctx *ctx, int32_t nshots, const double *f0_dev,
                          const double *f1_dev, fga_beams *beams);
/* Step 2: nsteps classical RK4 steps of the ray, dynamic ray tracing and
 * amplitude equations, in place.                                           */
fga_status fga3_propagate(fga3_ctx *ctx, fga_beams *beams, int32_t nshots, int32_t nsteps);
/* Step 3: u_dev[nshots][n3][n2][n1] = Re of the recons eq. over the boxes
 * (overwritten).                                                           */
fga_status fga3_reconstruct(fga3_ctx *ctx, const fga_beams *beams, int32_t nshots,
                            double *u_dev);
fga_status fga3_sync_status(fga3_ctx *ctx, int64_t *needed);
const char *fga3_last_error(const fga3_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FGA_H */
