// Internal declarations of the gfx950 FGA library: the context, launch
// helpers, and the device-side cubic B-spline velocity interpolant.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fga.h"

#define FGA_STATUS_CAPACITY 1
#define FGA_STATUS_NUMERIC 2

struct fga_ctx {
    fga_grid g;
    fga_params p;
    int prec;
    int max_shots;
    hipStream_t stream;
    int dev;
    int num_cu;

    // FBI box and reconstruction window half-widths (cells)
    int R1, R2, W1, W2;
    int Rw1, Rw2;
    double norm;           // w / (2 pi eps)^3

    double *c;             // velocity samples [n2][n1]
    double *cpad;          // the same with a replicated halo of FGA_VPAD cells
    double *ccoef;         // bicubic coefficients of every knot cell (16 per cell)
    bool have_c;

    // FBI workspaces
    void *E1t;             // [W1][np1] complex (pass-1 kernel table, m-major)
    void *E2;              // [np2][W2] complex (pass-2 kernel table)
    void *T;               // [nshots*nfj][n2][nq1*np1] complex
    void *Psi;             // [nshots*nfj][nq2][np2][nq1*np1] complex
    size_t T_bytes, Psi_bytes;
    double *cq;            // c(q) [nq2][nq1]
    unsigned long long *maxbits;   // per-shot max |psi| (double bits)
    unsigned *wmax;        // per-shot max |C a| (FP32 bits), FGA_MIXED_SPLIT splat
    unsigned *tmax;        // per (shot, part) max |Re T|, |Im T| (FP32 bits), split pass 2
    int64_t *blk;          // per-block counts / offsets of the compaction
    size_t blk_elems;

    // reconstruction workspaces: per-split partial sums, per-beam records
    double *partial;
    size_t partial_bytes;
    void *srec, *sbox;
    size_t srec_bytes, sbox_bytes;
    void *trace_part;      // per-split partial receiver sums
    size_t trace_part_bytes;
    void *bin;             // beam -> tile binning of the mixed splat
    size_t bin_bytes;

    // adjoint workspaces and the branch count of the last decomposition
    void *adj_scratch, *adj_psib;
    size_t adj_scratch_bytes, adj_psib_bytes;
    void *rec_shape;       // [4] ints: receivers one run of a row? (first column, row)
    size_t rec_shape_bytes;
    void *E1tt;            // [np1][W1] complex: pass-1 table, l-major (transposed pass 1)
    size_t E1tt_bytes;
    int last_nfj, last_nshots;

    // deterministic gradient: per-beam dJ/dc logs, the sort and cell
    // reductions, per-beam c(q) cotangents, a copy of an initial cotangent;
    // det_R is the log length per beam found sufficient so far
    void *det_log, *det_sort, *det_cell, *det_cqc, *det_lam;
    size_t det_log_bytes, det_sort_bytes, det_cell_bytes, det_cqc_bytes, det_lam_bytes;
    int det_R;

    // sticky device status: [0] flags, [1] needed capacity
    int64_t *status;

    // splat work split: target wavefronts (mixed) or workgroups (FP64) per
    // CU; 0 = built-in default, set by fga_autotune
    int splat_units_per_cu;

    // graph capture / replay of the whole forward
    bool capturing;
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    bool graph_stale;      // a workspace the graph uses was freed since capture

    // this device's copy of the library's static scratch array (fga_trace_noalloc)
    void *noalloc_scratch;

    char err[512];
};

fga_status fga_fail(fga_ctx *ctx, fga_status st, const char *fmt, ...);
fga_status fga_hip_check(fga_ctx *ctx, hipError_t e, const char *what);
fga_status fga_ensure(fga_ctx *ctx, void **buf, size_t *have, size_t need, const char *what);

#define FGA_HIP(ctx, call)                                                       \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) return fga_hip_check((ctx), e_, #call);            \
    } while (0)

// Stage launchers (defined in the stage sources)
fga_status fga_launch_decompose(fga_ctx *ctx, int nshots, const double *f0,
                                const double *f1, fga_beams *beams);
fga_status fga_launch_propagate(fga_ctx *ctx, fga_beams *beams, int nshots, int nsteps,
                                double *ckpt);
fga_status fga_launch_reconstruct(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                  double *u);
// Classify the receiver list on the device (no synchronisation): *shape
// receives a device pointer to {run, first column, row, run traced per beam}
// with run = 1 when rec[r] = rec[0] + r all lie in rec[0]'s row.
fga_status fga_rec_shape(fga_ctx *ctx, const int32_t *rec, int nrec, const int **shape);
// the same into a caller-given device buffer of 4 ints (no allocation)
fga_status fga_rec_shape_into(fga_ctx *ctx, const int32_t *rec, int nrec, int *shape);
fga_status fga_launch_trace_points(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                   const int32_t *rec, int nrec, double *out,
                                   int64_t out_stride_shot, const int *shape);
// work splits of the receiver sums (each split writes nshots * nrec partial
// sums), and the launch into caller-given partial sums (no allocation)
int fga_trace_splits(const fga_ctx *ctx, int nshots, int nrec);
fga_status fga_launch_trace_points_into(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                        const int32_t *rec, int nrec, double *out,
                                        int64_t out_stride_shot, const int *shape, double *part,
                                        int nsplit);

fga_status fga_launch_trace_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                    const int32_t *rec, int nrec, int rec_every, int nrec_t,
                                    const double *ckpt, const double *gtr, double *dc,
                                    double *gcoef);
fga_status fga_launch_rk4_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                  const int32_t *rec, int nrec, int rec_every, int nrec_t,
                                  const double *ckpt, const double *gtr, double *dc,
                                  double *gcoef, const double *lam0, double *lam_out);
fga_status fga_launch_reconstruct_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                          const double *du, double *dstate, double *dcoef);
// deterministic mode: (nb, total records, longest log) of the logs of the
// last adjoint kernel (synchronises), and the fixed-order reduction into dc
fga_status fga_det_stats(fga_ctx *ctx, const fga_beams *beams, int nshots, int R,
                         int64_t out[3]);
fga_status fga_det_reduce(fga_ctx *ctx, int64_t cap, int R, int64_t nb, int64_t total,
                          double *dc);
fga_status fga_launch_decompose_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                        const double *gcoef, double *df0, double *df1,
                                        double *dc);

static inline int fga_halfwidth(double eps, double tau, double d)
{
    return (int)ceil(sqrt(2.0 * eps * log(1.0 / tau)) / d);
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// The velocity samples are stored with a halo of FGA_VPAD replicated edge
// values on every side, so the four B-spline knots of any point whose knot
// index is first clamped to [-4, n + 4] are in range without per-tap
// clamping, and taps of one row are consecutive doubles.
#define FGA_VPAD 6

struct VelGrid {
    const double *c;      // padded samples, row length ld, origin at [FGA_VPAD][FGA_VPAD]
    const double *coef;   // per knot cell polynomial coefficients (vel_cell_coef)
    int n1, n2, ld;
    double o1, o2, inv_d1, inv_d2;
};

// Knot cells i1 in [-4, n1 + 3], i2 in [-4, n2 + 3] (see vel_cell): the
// coefficient table holds (n1 + 8) (n2 + 8) cells of 16 doubles.
#define FGA_VCELL_PAD 4
__host__ __device__ static inline int64_t fga_vcells(int n1, int n2)
{
    return (int64_t)(n1 + 2 * FGA_VCELL_PAD) * (n2 + 2 * FGA_VCELL_PAD);
}

// Cubic B-spline weights of the four knots floor(t)-1 .. floor(t)+2 and their
// first and second derivatives in t, for fractional part f in [0, 1).
__device__ __forceinline__ void bspline_w(double f, double w[4], double dw[4], double ddw[4])
{
    double g = 1.0 - f;
    double f2 = f * f, g2 = g * g;
    w[0] = g2 * g * (1.0 / 6.0);
    w[1] = (2.0 / 3.0) - f2 + 0.5 * f2 * f;
    w[2] = (2.0 / 3.0) - g2 + 0.5 * g2 * g;
    w[3] = f2 * f * (1.0 / 6.0);
    dw[0] = -0.5 * g2;
    dw[1] = -2.0 * f + 1.5 * f2;
    dw[2] = 2.0 * g - 1.5 * g2;
    dw[3] = 0.5 * f2;
    ddw[0] = g;
    ddw[1] = -2.0 + 3.0 * f;
    ddw[2] = -2.0 + 3.0 * g;
    ddw[3] = f;
}

// Knot cell of the B-spline evaluation at (x1, x2): the clamped index of the
// cell holding the point and the fractional offsets inside it.  Four or more
// cells outside the grid every knot reads the edge value, so clamping the
// index to [-4, n + 3] keeps the 4 x 4 taps inside the halo.
struct VelCell {
    int i1, i2;
    double f1, f2;
};

__device__ __forceinline__ VelCell vel_cell(const VelGrid &V, double x1, double x2)
{
    double t1 = (x1 - V.o1) * V.inv_d1;
    double t2 = (x2 - V.o2) * V.inv_d2;
    double fl1 = floor(t1), fl2 = floor(t2);
    VelCell k;
    k.f1 = t1 - fl1;
    k.f2 = t2 - fl2;
    k.i1 = (int)fmin(fmax(fl1, -4.0), (double)V.n1 + 3.0);
    k.i2 = (int)fmin(fmax(fl2, -4.0), (double)V.n2 + 3.0);
    return k;
}

// first of the 4 x 4 taps (row kz starts kz * V.ld further on)
__device__ __forceinline__ const double *vel_taps(const VelGrid &V, const VelCell &k)
{
    return V.c + (size_t)(k.i2 - 1 + FGA_VPAD) * V.ld + (k.i1 - 1 + FGA_VPAD);
}

// c, grad c and the Hessian (c11, c12, c22) of the clamped cubic B-spline
// from the taps of the cell; row(kz, v) fills v[0..3] with tap row kz.
template <class Rows>
__device__ __forceinline__ void vel_combine(const VelGrid &V, const VelCell &k, Rows row,
                                            double &c, double &c1, double &c2, double &c11,
                                            double &c12, double &c22)
{
    double wx[4], dwx[4], ddwx[4], wz[4], dwz[4], ddwz[4];
    bspline_w(k.f1, wx, dwx, ddwx);
    bspline_w(k.f2, wz, dwz, ddwz);
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
        double v[4];
        row(kz, v);
        double a0 = wx[0] * v[0] + wx[1] * v[1] + wx[2] * v[2] + wx[3] * v[3];
        double a1 = dwx[0] * v[0] + dwx[1] * v[1] + dwx[2] * v[2] + dwx[3] * v[3];
        double a2 = ddwx[0] * v[0] + ddwx[1] * v[1] + ddwx[2] * v[2] + ddwx[3] * v[3];
        s0 += wz[kz] * a0;
        s1 += wz[kz] * a1;
        s2 += dwz[kz] * a0;
        s3 += wz[kz] * a2;
        s4 += dwz[kz] * a1;
        s5 += ddwz[kz] * a0;
    }
    c = s0;
    c1 = s1 * V.inv_d1;
    c2 = s2 * V.inv_d2;
    c11 = s3 * V.inv_d1 * V.inv_d1;
    c12 = s4 * V.inv_d1 * V.inv_d2;
    c22 = s5 * V.inv_d2 * V.inv_d2;
}

// c, grad c and the Hessian of the clamped cubic B-spline at (x1, x2), taps
// read from the padded samples.
__device__ __forceinline__ void vel_eval(const VelGrid &V, double x1, double x2, double &c,
                                         double &c1, double &c2, double &c11, double &c12,
                                         double &c22)
{
    const VelCell k = vel_cell(V, x1, x2);
    const double *base = vel_taps(V, k);
    vel_combine(
        V, k,
        [&](int kz, double *v) {
            const double *r = base + kz * V.ld;
            v[0] = r[0];
            v[1] = r[1];
            v[2] = r[2];
            v[3] = r[3];
        },
        c, c1, c2, c11, c12, c22);
}

// Inside one knot cell the clamped cubic B-spline is the bicubic polynomial
// c = sum_{a,b} C[b][a] f1^a f2^b of the fractional offsets.  The table holds
// C[b][a] at entry 4 b + a of the cell's 16 doubles (one 128-byte line).
__device__ __forceinline__ const double *vel_cell_coef(const VelGrid &V, const VelCell &k)
{
    return V.coef + ((int64_t)(k.i2 + FGA_VCELL_PAD) * (V.n1 + 2 * FGA_VCELL_PAD) +
                     (k.i1 + FGA_VCELL_PAD)) * 16;
}

// c, grad c and the Hessian from the cell's coefficients C[b][a] by Horner's
// rule: first in f2 for every power of f1 (value, first and half the second
// derivative), then in f1.  The derivative forms carry their factors in the
// multipliers, e.g. 3 C3 f^2 + 2 C2 f + C1 = (C3 (1.5 f) + C2)(2 f) + C1 and
// (6 C3 f + 2 C2) / 2 = C3 (3 f) + C2, so every step is one FMA; the halves
// are doubled in the final scaling.
__device__ __forceinline__ void vel_poly(const VelGrid &V, const VelCell &k,
                                         const double C[4][4], double &c, double &c1, double &c2,
                                         double &c11, double &c12, double &c22)
{
    const double f1 = k.f1, f2 = k.f2;
    const double f2h = 1.5 * f2, f2d = 2.0 * f2, f2t = 3.0 * f2;
    double q[4], q1[4], q2h[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        q[a] = fma(fma(fma(C[3][a], f2, C[2][a]), f2, C[1][a]), f2, C[0][a]);
        q1[a] = fma(fma(C[3][a], f2h, C[2][a]), f2d, C[1][a]);
        q2h[a] = fma(C[3][a], f2t, C[2][a]);
    }
    const double f1h = 1.5 * f1, f1d = 2.0 * f1, f1t = 3.0 * f1;
    c = fma(fma(fma(q[3], f1, q[2]), f1, q[1]), f1, q[0]);
    const double d1 = fma(fma(q[3], f1h, q[2]), f1d, q[1]);
    const double d11h = fma(q[3], f1t, q[2]);
    const double d2 = fma(fma(fma(q1[3], f1, q1[2]), f1, q1[1]), f1, q1[0]);
    const double d12 = fma(fma(q1[3], f1h, q1[2]), f1d, q1[1]);
    const double d22h = fma(fma(fma(q2h[3], f1, q2h[2]), f1, q2h[1]), f1, q2h[0]);
    c1 = d1 * V.inv_d1;
    c2 = d2 * V.inv_d2;
    c11 = d11h * (2.0 * V.inv_d1 * V.inv_d1);
    c12 = d12 * (V.inv_d1 * V.inv_d2);
    c22 = d22h * (2.0 * V.inv_d2 * V.inv_d2);
}

// c, grad c and the Hessian at (x1, x2) from the knot cell's coefficient line
// (the same polynomial, and the same rounding, as the RK4 kernel's LDS path)
__device__ __forceinline__ void vel_eval_coef(const VelGrid &V, double x1, double x2, double &c,
                                              double &c1, double &c2, double &c11, double &c12,
                                              double &c22)
{
    const VelCell k = vel_cell(V, x1, x2);
    const double2 *line = reinterpret_cast<const double2 *>(vel_cell_coef(V, k));
    double C[4][4];
#pragma unroll
    for (int sl = 0; sl < 8; ++sl) {
        const double2 v = line[sl];
        C[sl >> 1][2 * (sl & 1)] = v.x;
        C[sl >> 1][2 * (sl & 1) + 1] = v.y;
    }
    vel_poly(V, k, C, c, c1, c2, c11, c12, c22);
}

// Truncation box of a Gaussian centred at Q: the nodes within Rw cells of the
// node nearest Q (floor(t + 1/2)), clipped to the grid.
struct BeamBox {
    int lo1, hi1, lo2, hi2;
};

__device__ __forceinline__ BeamBox beam_box(double Q1, double Q2, double o1, double o2,
                                            double d1, double d2, int Rw1, int Rw2, int n1,
                                            int n2)
{
    // nearest node by floor(t + 1/2); far-away centres are clamped before the
    // integer conversion (their boxes miss the grid either way)
    double t1 = fmin(fmax(floor((Q1 - o1) / d1 + 0.5), -1e8), 1e8);
    double t2 = fmin(fmax(floor((Q2 - o2) / d2 + 0.5), -1e8), 1e8);
    int c1 = (int)t1, c2 = (int)t2;
    BeamBox b;
    b.lo1 = max(c1 - Rw1, 0);
    b.hi1 = min(c1 + Rw1, n1 - 1);
    b.lo2 = max(c2 - Rw2, 0);
    b.hi2 = min(c2 + Rw2, n2 - 1);
    return b;
}

static inline VelGrid fga_velgrid(const fga_ctx *ctx)
{
    VelGrid V;
    V.c = ctx->cpad;
    V.coef = ctx->ccoef;
    V.n1 = ctx->g.n1;
    V.n2 = ctx->g.n2;
    V.ld = ctx->g.n1 + 2 * FGA_VPAD;
    V.o1 = ctx->g.o1;
    V.o2 = ctx->g.o2;
    V.inv_d1 = 1.0 / ctx->g.d1;
    V.inv_d2 = 1.0 / ctx->g.d2;
    return V;
}
