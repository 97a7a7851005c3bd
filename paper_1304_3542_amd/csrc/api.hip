// C ABI entry points: argument validation, context and workspace management.
// The stage kernels live in fbi.hip, propagate.hip and reconstruct.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "fga_internal.h"

static char g_create_err[512] = "";

// Scratch of fga_trace_noalloc: one static array per device (each GPU the
// library runs on holds its own copy until the process ends).  Host code never
// uses this name as an address: fga_create looks up the device address once
// per device and every launch takes that pointer.
static __device__ __align__(256) unsigned char scratch[FGA_NOALLOC_SCRATCH_BYTES];

#define FGA_MAX_DEVICES 64
static void *g_scratch_ptr[FGA_MAX_DEVICES];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device (dev), looked up on
// the first context created there.
static fga_status scratch_address(int dev, void **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= FGA_MAX_DEVICES) return FGA_OK;   // variant unavailable there
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fga_fail(nullptr, FGA_EHIP, "hipGetSymbolAddress(scratch): %s",
                            hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FGA_OK;
}

fga_status fga_fail(fga_ctx *ctx, fga_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx ? ctx->err : g_create_err, 512, fmt, ap);
    va_end(ap);
    return st;
}

fga_status fga_hip_check(fga_ctx *ctx, hipError_t e, const char *what)
{
    if (e == hipSuccess) return FGA_OK;
    return fga_fail(ctx, e == hipErrorOutOfMemory ? FGA_ENOMEM : FGA_EHIP, "%s: %s", what,
                    hipGetErrorString(e));
}

fga_status fga_ensure(fga_ctx *ctx, void **buf, size_t *have, size_t need, const char *what)
{
    if (*have >= need && *buf) return FGA_OK;
    if (ctx->capturing)
        return fga_fail(ctx, FGA_ESTATE, "%s would need an allocation during graph capture", what);
    if (*buf) {
        // the old buffer may still be read by queued work
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return fga_hip_check(ctx, e, "hipStreamSynchronize");
        (void)hipFree(*buf);
        *buf = nullptr;
        *have = 0;
        // a captured graph holds the freed address: refuse to replay it
        if (ctx->graph_exec) ctx->graph_stale = true;
    }
    hipError_t e = hipMalloc(buf, need);
    if (e != hipSuccess) {
        *buf = nullptr;
        return fga_fail(ctx, FGA_ENOMEM, "hipMalloc(%zu bytes) for %s failed: %s", need, what,
                        hipGetErrorString(e));
    }
    *have = need;
    return FGA_OK;
}

static fga_status check_params(fga_ctx *ctx, const fga_grid *g, const fga_params *p)
{
    // node indices of truncation boxes are stored as 16-bit integers, with
    // n itself marking an empty box
    if (g->n1 < 4 || g->n2 < 4 || g->n1 > FGA_MAX_N || g->n2 > FGA_MAX_N)
        return fga_fail(ctx, FGA_EINVAL, "grid size %d x %d outside [4, %d]", g->n1, g->n2,
                        FGA_MAX_N);
    if (!(g->d1 > 0) || !(g->d2 > 0) || !isfinite(g->o1) || !isfinite(g->o2))
        return fga_fail(ctx, FGA_EINVAL, "grid spacing must be positive and origin finite");
    if (!(p->eps > 0) || !isfinite(p->eps))
        return fga_fail(ctx, FGA_EINVAL, "eps must be positive");
    if (p->nq1 < 1 || p->nq2 < 1 || p->qs1 < 1 || p->qs2 < 1)
        return fga_fail(ctx, FGA_EINVAL, "q-mesh sizes and strides must be >= 1");
    if (p->qb1 < 0 || p->qb2 < 0 || p->qb1 + (int64_t)(p->nq1 - 1) * p->qs1 >= g->n1 ||
        p->qb2 + (int64_t)(p->nq2 - 1) * p->qs2 >= g->n2)
        return fga_fail(ctx, FGA_EINVAL, "q-mesh leaves the grid");
    if (p->np1 < 2 || p->np2 < 2 || (p->np1 & 1) || (p->np2 & 1) || p->np1 > 4096 ||
        p->np2 > 4096)
        return fga_fail(ctx, FGA_EINVAL, "p-mesh sizes must be even, in [2, 4096]");
    if (!(p->dp1 > 0) || !(p->dp2 > 0))
        return fga_fail(ctx, FGA_EINVAL, "p-mesh spacing must be positive");
    if (!(p->tau >= 0 && p->tau <= 1))
        return fga_fail(ctx, FGA_EINVAL, "tau must lie in [0, 1]");
    if (!(p->tau_fbi > 0 && p->tau_fbi < 1) || !(p->tau_win > 0 && p->tau_win < 1))
        return fga_fail(ctx, FGA_EINVAL, "tau_fbi and tau_win must lie in (0, 1)");
    if (!(p->dt > 0) || !isfinite(p->dt)) return fga_fail(ctx, FGA_EINVAL, "dt must be positive");
    if (p->top_n < 0) return fga_fail(ctx, FGA_EINVAL, "top_n must be >= 0");
    if (p->amp_closed != 0 && p->amp_closed != 1)
        return fga_fail(ctx, FGA_EINVAL, "amp_closed must be 0 or 1");
    if (p->dz_divided != 0 && p->dz_divided != 1)
        return fga_fail(ctx, FGA_EINVAL, "dz_divided must be 0 or 1");
    if (p->dz_divided && !p->amp_closed)
        return fga_fail(ctx, FGA_EINVAL,
                        "dz_divided = 1 takes the closed-form amplitude (amp_closed = 1)");
    if (p->dz_divided && !(p->dz_scale > 0 && isfinite(p->dz_scale)))
        return fga_fail(ctx, FGA_EINVAL, "dz_scale must be positive");
    if (p->deterministic != 0 && p->deterministic != 1)
        return fga_fail(ctx, FGA_EINVAL, "deterministic must be 0 or 1");
    if (p->grad_log < -1)
        return fga_fail(ctx, FGA_EINVAL, "grad_log must be -1, 0 or positive");
    if (p->ckpt_every_step != 0 && p->ckpt_every_step != 1)
        return fga_fail(ctx, FGA_EINVAL, "ckpt_every_step must be 0 or 1");
    if (p->ckpt_every_step && (p->amp_closed || p->dz_divided))
        return fga_fail(ctx, FGA_EINVAL,
                        "ckpt_every_step requires the integrated amplitude (amp_closed = 0)");
    int R1 = fga_halfwidth(p->eps, p->tau_fbi, g->d1);
    int R2 = fga_halfwidth(p->eps, p->tau_fbi, g->d2);
    if (R1 > 8192 || R2 > 8192)
        return fga_fail(ctx, FGA_EINVAL, "FBI box of %d x %d cells is too large", 2 * R1 + 1,
                        2 * R2 + 1);
    return FGA_OK;
}

extern "C" fga_status fga_create(fga_ctx **out, const fga_grid *g, const fga_params *p,
                                 int32_t precision, int32_t max_shots, void *stream)
{
    if (!out || !g || !p) return fga_fail(nullptr, FGA_EINVAL, "null argument to fga_create");
    *out = nullptr;
    if (precision != FGA_FP64 && precision != FGA_MIXED && precision != FGA_MIXED_SPLIT)
        return fga_fail(nullptr, FGA_EINVAL, "unknown precision %d", precision);
    if (max_shots < 1 || max_shots > 65535)
        return fga_fail(nullptr, FGA_EINVAL, "max_shots must lie in [1, 65535]");
    fga_status st = check_params(nullptr, g, p);
    if (st != FGA_OK) return st;

    fga_ctx *ctx = (fga_ctx *)calloc(1, sizeof(fga_ctx));
    if (!ctx) return fga_fail(nullptr, FGA_ENOMEM, "host allocation failed");
    ctx->g = *g;
    ctx->p = *p;
    ctx->prec = precision;
    ctx->max_shots = max_shots;
    ctx->stream = (hipStream_t)stream;
    ctx->R1 = fga_halfwidth(p->eps, p->tau_fbi, g->d1);
    ctx->R2 = fga_halfwidth(p->eps, p->tau_fbi, g->d2);
    ctx->W1 = 2 * ctx->R1 + 1;
    ctx->W2 = 2 * ctx->R2 + 1;
    ctx->Rw1 = fga_halfwidth(p->eps, p->tau_win, g->d1);
    ctx->Rw2 = fga_halfwidth(p->eps, p->tau_win, g->d2);
    double w = (p->qs1 * g->d1) * (p->qs2 * g->d2) * p->dp1 * p->dp2;
    double tpe = 2.0 * M_PI * p->eps;
    ctx->norm = w / (tpe * tpe * tpe);

    hipError_t e = hipGetDevice(&ctx->dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, ctx->dev);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->c, sizeof(double) * g->n1 * g->n2);
    if (e == hipSuccess)
        e = hipMalloc((void **)&ctx->cpad, sizeof(double) * (g->n1 + 2 * FGA_VPAD) *
                                               (g->n2 + 2 * FGA_VPAD));
    if (e == hipSuccess)
        e = hipMalloc((void **)&ctx->ccoef, sizeof(double) * 16 * fga_vcells(g->n1, g->n2));
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->status, 2 * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->cq, sizeof(double) * p->nq1 * p->nq2);
    if (e == hipSuccess)
        e = hipMalloc((void **)&ctx->maxbits, sizeof(unsigned long long) * max_shots);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->wmax, sizeof(unsigned) * max_shots);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->tmax, sizeof(unsigned) * 2 * max_shots);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->status, 0, 2 * sizeof(int64_t), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        fga_fail(nullptr, FGA_EHIP, "fga_create: %s", hipGetErrorString(e));
        fga_destroy(ctx);
        return FGA_EHIP;
    }
    st = scratch_address(ctx->dev, &ctx->noalloc_scratch);
    if (st != FGA_OK) {
        fga_destroy(ctx);
        return st;
    }
    *out = ctx;
    return FGA_OK;
}

extern "C" fga_status fga_destroy(fga_ctx *ctx)
{
    if (!ctx) return FGA_OK;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    void *bufs[] = {ctx->c, ctx->cpad, ctx->ccoef, ctx->status, ctx->cq, ctx->maxbits, ctx->wmax, ctx->tmax, ctx->E1t, ctx->E2,
                    ctx->T, ctx->Psi, ctx->blk, ctx->partial, ctx->srec, ctx->sbox,
                    ctx->adj_scratch, ctx->adj_psib, ctx->rec_shape, ctx->E1tt, ctx->trace_part, ctx->bin,
                    ctx->det_log, ctx->det_sort, ctx->det_cell, ctx->det_cqc, ctx->det_lam};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    free(ctx);
    return FGA_OK;
}

extern "C" fga_status fga_set_stream(fga_ctx *ctx, void *stream)
{
    if (!ctx) return FGA_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return FGA_OK;
}

// Checks c > 0 and finite, and writes the padded copy (edge values
// replicated into the halo, i.e. clamped indices).
__global__ void k_pad_velocity(const double *c, int n1, int n2, double *cpad, int64_t *status)
{
    int ld = n1 + 2 * FGA_VPAD, rows = n2 + 2 * FGA_VPAD;
    int64_t n = (int64_t)ld * rows;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int r = (int)(i / ld), q = (int)(i % ld);
        int i2 = min(max(r - FGA_VPAD, 0), n2 - 1), i1 = min(max(q - FGA_VPAD, 0), n1 - 1);
        double v = c[(size_t)i2 * n1 + i1];
        if (!(v > 0.0) || !isfinite(v)) atomicOr((unsigned long long *)status, FGA_STATUS_NUMERIC);
        cpad[i] = v;
    }
}

// Bicubic coefficients of every knot cell: with the uniform B-spline basis
// in powers of the offset f, w_k(f) = sum_a M[k][a] f^a / 6, the cell's
// polynomial is C[b][a] = sum_{kz,kx} M[kz][b] M[kx][a] v[kz][kx] / 36 over
// its 4 x 4 taps v (row kz along axis 2).
__global__ void k_vel_coef(const double *cpad, int n1, int n2, double *coef)
{
    const double M[4][4] = {{1, -3, 3, -1}, {4, 0, -6, 3}, {1, 3, 3, -3}, {0, 0, 0, 1}};
    const int ld = n1 + 2 * FGA_VPAD, nc1 = n1 + 2 * FGA_VCELL_PAD;
    const int64_t ncell = fga_vcells(n1, n2);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int i1 = (int)(i % nc1) - FGA_VCELL_PAD, i2 = (int)(i / nc1) - FGA_VCELL_PAD;
        const double *base = cpad + (size_t)(i2 - 1 + FGA_VPAD) * ld + (i1 - 1 + FGA_VPAD);
        double T[4][4];   // T[kz][a] = sum_kx v[kz][kx] M[kx][a]
#pragma unroll
        for (int kz = 0; kz < 4; ++kz)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double t = 0.0;
#pragma unroll
                for (int kx = 0; kx < 4; ++kx) t += base[kz * ld + kx] * M[kx][a];
                T[kz][a] = t;
            }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double t = 0.0;
#pragma unroll
                for (int kz = 0; kz < 4; ++kz) t += M[kz][b] * T[kz][a];
                coef[i * 16 + 4 * b + a] = t * (1.0 / 36.0);
            }
    }
}

extern "C" fga_status fga_set_velocity(fga_ctx *ctx, const double *c_dev)
{
    if (!ctx || !c_dev) return ctx ? fga_fail(ctx, FGA_EINVAL, "null velocity") : FGA_EINVAL;
    size_t n = (size_t)ctx->g.n1 * ctx->g.n2;
    FGA_HIP(ctx, hipMemcpyAsync(ctx->c, c_dev, n * sizeof(double), hipMemcpyDeviceToDevice,
                                ctx->stream));
    hipLaunchKernelGGL(k_pad_velocity, dim3(256), dim3(256), 0, ctx->stream, ctx->c,
                       ctx->g.n1, ctx->g.n2, ctx->cpad, ctx->status);
    hipLaunchKernelGGL(k_vel_coef, dim3(1024), dim3(256), 0, ctx->stream, ctx->cpad, ctx->g.n1,
                       ctx->g.n2, ctx->ccoef);
    FGA_HIP(ctx, hipGetLastError());
    ctx->have_c = true;
    return FGA_OK;
}

static fga_status check_beams(fga_ctx *ctx, const fga_beams *b)
{
    if (!b || !b->f || !b->id || !b->offsets || b->capacity < 1)
        return fga_fail(ctx, FGA_EINVAL, "beam buffers must be non-null with capacity >= 1");
    return FGA_OK;
}

extern "C" fga_status fga_decompose(fga_ctx *ctx, int32_t nshots, const double *f0,
                                    const double *f1, fga_beams *beams)
{
    if (!ctx) return FGA_EINVAL;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!f0) return fga_fail(ctx, FGA_EINVAL, "f0 is null");
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    return fga_launch_decompose(ctx, nshots, f0, f1, beams);
}

extern "C" fga_status fga_propagate(fga_ctx *ctx, fga_beams *beams, int32_t nshots,
                                    int32_t nsteps)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (nsteps < 0) return fga_fail(ctx, FGA_EINVAL, "nsteps must be >= 0");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    if (nsteps == 0) return FGA_OK;
    return fga_launch_propagate(ctx, beams, nshots, nsteps, nullptr);
}

extern "C" fga_status fga_reconstruct(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                      double *u)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!u) return fga_fail(ctx, FGA_EINVAL, "u is null");
    return fga_launch_reconstruct(ctx, beams, nshots, u);
}

extern "C" fga_status fga_trace(fga_ctx *ctx, fga_beams *beams, int32_t nshots,
                                const int32_t *rec, int32_t nrec, int32_t rec_every,
                                int32_t nrec_t, double *traces, double *ckpt)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!rec || nrec < 1 || rec_every < 1 || nrec_t < 1 || !traces)
        return fga_fail(ctx, FGA_EINVAL, "bad receiver arguments");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    const int *shape = nullptr;
    st = fga_rec_shape(ctx, rec, nrec, &shape);
    if (st != FGA_OK) return st;
    for (int k = 0; k < nrec_t; ++k) {
        const size_t per = ctx->p.ckpt_every_step ? (size_t)rec_every : 1;
        double *ck = ckpt ? ckpt + (size_t)k * per * FGA_NSTATE * beams->capacity : nullptr;
        st = fga_launch_propagate(ctx, beams, nshots, rec_every, ck);
        if (st != FGA_OK) return st;
        st = fga_launch_trace_points(ctx, beams, nshots, rec, nrec, traces + (size_t)k * nrec,
                                     (int64_t)nrec_t * nrec, shape);
        if (st != FGA_OK) return st;
    }
    return FGA_OK;
}

extern "C" fga_status fga_trace_noalloc(fga_ctx *ctx, fga_beams *beams, int32_t nshots,
                                        const int32_t *rec, int32_t nrec, int32_t rec_every,
                                        int32_t nrec_t, double *traces, double *ckpt)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!rec || nrec < 1 || rec_every < 1 || nrec_t < 1 || !traces)
        return fga_fail(ctx, FGA_EINVAL, "bad receiver arguments");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    if (!ctx->noalloc_scratch)
        return fga_fail(ctx, FGA_ESTATE, "no static scratch on device %d", ctx->dev);
    // layout: the receiver classification (4 ints) in the first 256 bytes,
    // then the partial sums [nshots][nsplit][nrec]; every entry is written
    // before it is read, so nothing needs clearing
    const size_t avail = FGA_NOALLOC_SCRATCH_BYTES - 256;
    const size_t per_split = (size_t)nshots * nrec * sizeof(double);
    if (per_split > avail)
        return fga_fail(ctx, FGA_EINVAL,
                        "fga_trace_noalloc: %d shots x %d receivers need %zu bytes of scratch, "
                        "above its %lld bytes",
                        nshots, nrec, per_split + 256, (long long)FGA_NOALLOC_SCRATCH_BYTES);
    int nsplit = fga_trace_splits(ctx, nshots, nrec);
    if ((size_t)nsplit * per_split > avail) nsplit = (int)(avail / per_split);
    int *shape = (int *)ctx->noalloc_scratch;
    double *part = (double *)((char *)ctx->noalloc_scratch + 256);
    st = fga_rec_shape_into(ctx, rec, nrec, shape);
    if (st != FGA_OK) return st;
    for (int k = 0; k < nrec_t; ++k) {
        const size_t per = ctx->p.ckpt_every_step ? (size_t)rec_every : 1;
        double *ck = ckpt ? ckpt + (size_t)k * per * FGA_NSTATE * beams->capacity : nullptr;
        st = fga_launch_propagate(ctx, beams, nshots, rec_every, ck);
        if (st != FGA_OK) return st;
        st = fga_launch_trace_points_into(ctx, beams, nshots, rec, nrec,
                                          traces + (size_t)k * nrec, (int64_t)nrec_t * nrec,
                                          shape, part, nsplit);
        if (st != FGA_OK) return st;
    }
    return FGA_OK;
}

extern "C" fga_status fga_trace_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                        const int32_t *rec, int32_t nrec, int32_t rec_every,
                                        int32_t nrec_t, const double *ckpt, const double *gtr,
                                        double *dc, double *gcoef)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!rec || nrec < 1 || rec_every < 1 || nrec_t < 1 || !ckpt || !gtr || !dc || !gcoef)
        return fga_fail(ctx, FGA_EINVAL, "bad trace-adjoint arguments");
    if (ctx->p.amp_closed)
        return fga_fail(ctx, FGA_EINVAL, "the trace adjoint needs the integrated amplitude");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    return fga_launch_trace_adjoint(ctx, beams, nshots, rec, nrec, rec_every, nrec_t, ckpt, gtr,
                                    dc, gcoef);
}

extern "C" fga_status fga_propagate_ckpt(fga_ctx *ctx, fga_beams *beams, int32_t nshots,
                                         int32_t seg, int32_t nseg, double *ckpt)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (seg < 1 || nseg < 1 || !ckpt)
        return fga_fail(ctx, FGA_EINVAL, "bad checkpoint arguments");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    const size_t per = ctx->p.ckpt_every_step ? (size_t)seg : 1;
    for (int k = 0; k < nseg; ++k) {
        st = fga_launch_propagate(ctx, beams, nshots, seg,
                                  ckpt + (size_t)k * per * FGA_NSTATE * beams->capacity);
        if (st != FGA_OK) return st;
    }
    return FGA_OK;
}

extern "C" fga_status fga_propagate_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                            int32_t seg, int32_t nseg, const double *ckpt,
                                            double *dstate, double *dc)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (seg < 1 || nseg < 1 || !ckpt || !dstate || !dc)
        return fga_fail(ctx, FGA_EINVAL, "bad propagate-adjoint arguments");
    if (ctx->p.amp_closed)
        return fga_fail(ctx, FGA_EINVAL, "the propagation adjoint needs the integrated amplitude");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    return fga_launch_rk4_adjoint(ctx, beams, nshots, nullptr, 0, seg, nseg, ckpt, nullptr, dc,
                                  nullptr, dstate, dstate);
}

extern "C" fga_status fga_reconstruct_adjoint(fga_ctx *ctx, const fga_beams *beams,
                                              int32_t nshots, const double *du, double *dstate,
                                              double *dcoef)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!du || !dstate || !dcoef)
        return fga_fail(ctx, FGA_EINVAL, "du, dstate and dcoef must be non-null");
    return fga_launch_reconstruct_adjoint(ctx, beams, nshots, du, dstate, dcoef);
}

extern "C" fga_status fga_decompose_adjoint(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                            const double *gcoef, double *df0, double *df1,
                                            double *dc)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    if (!gcoef || !df0) return fga_fail(ctx, FGA_EINVAL, "gcoef and df0 must be non-null");
    if (!ctx->Psi || ctx->last_nfj < 1)
        return fga_fail(ctx, FGA_ESTATE, "fga_decompose has not run on this context");
    if (nshots != ctx->last_nshots)
        return fga_fail(ctx, FGA_EINVAL, "nshots %d differs from the last fga_decompose (%d)",
                        nshots, ctx->last_nshots);
    if (ctx->last_nfj == 2 && (!df1 || !dc))
        return fga_fail(ctx, FGA_EINVAL, "the decomposition used f1: df1 and dc are required");
    return fga_launch_decompose_adjoint(ctx, beams, nshots, gcoef, df0, df1, dc);
}

// One forward pass (decompose, propagate, reconstruct) of nshots shots.
static fga_status forward_pass(fga_ctx *ctx, int nshots, const double *f0, const double *f1,
                               fga_beams *beams, int nsteps, double *u)
{
    fga_status st = fga_launch_decompose(ctx, nshots, f0, f1, beams);
    if (st == FGA_OK && nsteps > 0) st = fga_launch_propagate(ctx, beams, nshots, nsteps, nullptr);
    if (st == FGA_OK) st = fga_launch_reconstruct(ctx, beams, nshots, u);
    return st;
}

extern "C" fga_status fga_graph_capture(fga_ctx *ctx, int32_t nshots, const double *f0,
                                        const double *f1, fga_beams *beams, int32_t nsteps,
                                        double *u)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots || !f0 || !u || nsteps < 0)
        return fga_fail(ctx, FGA_EINVAL, "bad graph-capture arguments");
    if (!ctx->have_c) return fga_fail(ctx, FGA_ESTATE, "fga_set_velocity was not called");
    // one eager pass on the context's stream sizes every workspace
    st = forward_pass(ctx, nshots, f0, f1, beams, nsteps, u);
    if (st != FGA_OK) return st;
    FGA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->graph_exec) {
        FGA_HIP(ctx, hipGraphExecDestroy(ctx->graph_exec));
        ctx->graph_exec = nullptr;
    }
    if (ctx->graph) {
        FGA_HIP(ctx, hipGraphDestroy(ctx->graph));
        ctx->graph = nullptr;
    }
    if (!ctx->cap_stream) FGA_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = forward_pass(ctx, nshots, f0, f1, beams, nsteps, u);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
        if (st == FGA_OK && e2 != hipSuccess) st = fga_hip_check(ctx, e2, "hipStreamEndCapture");
        if (st == FGA_OK) {
            ctx->graph = g;
            hipError_t e3 = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
            if (e3 != hipSuccess) st = fga_hip_check(ctx, e3, "hipGraphInstantiate");
            else ctx->graph_stale = false;
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    } else {
        st = fga_hip_check(ctx, e, "hipStreamBeginCapture");
    }
    ctx->capturing = false;
    ctx->stream = user;
    return st;
}

extern "C" fga_status fga_graph_launch(fga_ctx *ctx)
{
    if (!ctx) return FGA_EINVAL;
    if (!ctx->graph_exec) return fga_fail(ctx, FGA_ESTATE, "no captured graph");
    if (ctx->graph_stale)
        return fga_fail(ctx, FGA_ESTATE,
                        "a workspace of the captured graph was reallocated by a later call; "
                        "capture again");
    FGA_HIP(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
    return FGA_OK;
}

// Times the reconstruction for a ladder of work splits on the given beams
// (which must be propagated already), keeps the fastest, and records it in
// a JSON-lines cache keyed by grid, window, precision and shot count.
extern "C" fga_status fga_autotune(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                   double *u, const char *cache_path, int32_t *chosen)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (nshots < 1 || nshots > ctx->max_shots || !u)
        return fga_fail(ctx, FGA_EINVAL, "bad autotune arguments");
    char key[256];
    snprintf(key, sizeof key, "%dx%d|Rw%dx%d|prec%d|shots%d|cu%d", ctx->g.n1, ctx->g.n2,
             ctx->Rw1, ctx->Rw2, ctx->prec, nshots, ctx->num_cu);
    if (cache_path) {
        FILE *fp = fopen(cache_path, "r");
        if (fp) {
            char line[512], k[256];
            int v;
            int found = 0;
            while (fgets(line, sizeof line, fp))
                if (sscanf(line, "{\"key\": \"%255[^\"]\", \"splat_units_per_cu\": %d}", k, &v) == 2 &&
                    strcmp(k, key) == 0) {
                    ctx->splat_units_per_cu = v;
                    found = 1;
                }
            fclose(fp);
            if (found) {
                if (chosen) *chosen = ctx->splat_units_per_cu;
                return FGA_OK;
            }
        }
    }
    const int mixed[] = {4, 8, 16, 32, 64, 128};
    const int fp64[] = {2, 4, 8, 16, 32, 64};
    const int *cand = ctx->prec != FGA_FP64 ? mixed : fp64;
    const int ncand = 6;
    hipEvent_t e0, e1;
    FGA_HIP(ctx, hipEventCreate(&e0));
    FGA_HIP(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    int best_v = 0;
    for (int i = 0; i < ncand && st == FGA_OK; ++i) {
        ctx->splat_units_per_cu = cand[i];
        st = fga_launch_reconstruct(ctx, beams, nshots, u);   // sizes the workspace
        if (st != FGA_OK) break;
        float tot = 0.f;
        for (int r = 0; r < 3 && st == FGA_OK; ++r) {
            (void)hipEventRecord(e0, ctx->stream);
            st = fga_launch_reconstruct(ctx, beams, nshots, u);
            (void)hipEventRecord(e1, ctx->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tot += ms;
        }
        if (tot < best) {
            best = tot;
            best_v = cand[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FGA_OK) return st;
    ctx->splat_units_per_cu = best_v;
    if (chosen) *chosen = best_v;
    if (cache_path) {
        FILE *fp = fopen(cache_path, "a");
        if (fp) {
            fprintf(fp, "{\"key\": \"%s\", \"splat_units_per_cu\": %d}\n", key, best_v);
            fclose(fp);
        }
    }
    return FGA_OK;
}

extern "C" fga_status fga_sync_status(fga_ctx *ctx, int64_t *needed)
{
    if (!ctx) return FGA_EINVAL;
    int64_t h[2] = {0, 0};
    FGA_HIP(ctx, hipMemcpyAsync(h, ctx->status, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    FGA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    FGA_HIP(ctx, hipMemsetAsync(ctx->status, 0, 2 * sizeof(int64_t), ctx->stream));
    FGA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (needed) *needed = h[1];
    if (h[0] & FGA_STATUS_NUMERIC)
        return fga_fail(ctx, FGA_ENUMERIC, "non-finite value or c <= 0 met on the device");
    if (h[0] & FGA_STATUS_CAPACITY)
        return fga_fail(ctx, FGA_ECAPACITY, "beam capacity exceeded: %lld beams needed",
                        (long long)h[1]);
    return FGA_OK;
}

extern "C" fga_status fga_copy_offsets(fga_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                       int64_t *host)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = check_beams(ctx, beams);
    if (st != FGA_OK) return st;
    if (!host || nshots < 1) return fga_fail(ctx, FGA_EINVAL, "bad arguments");
    FGA_HIP(ctx, hipMemcpyAsync(host, beams->offsets, sizeof(int64_t) * (nshots + 1),
                                hipMemcpyDeviceToHost, ctx->stream));
    FGA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FGA_OK;
}

extern "C" const char *fga_last_error(const fga_ctx *ctx)
{
    return ctx ? ctx->err : g_create_err;
}
