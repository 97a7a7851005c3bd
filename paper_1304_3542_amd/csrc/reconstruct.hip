// Step 3 of the FGA algorithm on gfx950: the frozen-Gaussian sum (recons eq.)
//   u(x) = Re sum_b C_b a_b e^{i S_b/eps} e^{i P_b.(x-Q_b)/eps - |x-Q_b|^2/(2 eps)}
// over the nodes of each beam's truncation box.  The Gaussian and the plane
// wave both factor over the two axes, so inside an output tile
//   term_b(x1, x2) = U_b(x1) V_b(x2),
//   U_b(x1) = C_b a_b e^{i(S_b + P1 r1)/eps - r1^2/(2 eps)},  r1 = x1 - Q1,
//   V_b(x2) = e^{i P2 r2/eps - r2^2/(2 eps)},                r2 = x2 - Q2,
// with U (V) set to zero outside the beam's box, and Re(U V) = Ur Vr - Ui Vi.
// A workgroup owns a 64 x 64 tile and one slice of a shot's beam list: it
// keeps the beams whose box meets the tile (order preserved), evaluates the
// 128 factors of each into LDS and accumulates the rank-one updates in
// registers.  Slices write private partial tiles that a second kernel adds
// in slice order, so the result is deterministic.
//
// FP64 path: factors and sums in double.  Mixed path: the phase is formed
// and reduced mod 2 pi in double, then sin/cos/exp and the sums run in FP32,
// and every 256 beams the FP32 partial sums are folded into FP64 ones.
#include <math.h>

#include "splat.h"

// FP64 splat.  A workgroup takes one 128 x 128 tile and one slice of its
// shot's beams; thread (tx, tz) owns the 8 x 8 nodes (X0 + tx + 16 i,
// Z0 + tz + 16 j).  The slice is scanned 256 beams at a time, the beams whose
// box meets the tile listed in order, and taken 16 at a time: their factors
//   U(x1) = C a e^{(i (S + P1 r1) - r1^2/2) / eps},  V(x2) = e^{(i P2 r2 - r2^2/2) / eps}
// at the tile's 128 + 128 coordinates (zero outside the box) go to LDS, and
// every thread adds Re(U V) = Ur Vr - Ui Vi to its 64 nodes.  The factors
// are formed in runs of 16 consecutive nodes, one direct evaluation at the
// run's first node in the box and then g(x + d) = g(x) rho(x),
// rho(x + d) = rho(x) e^{-d^2/eps} (exact identities of the Gaussian).

__global__ void __launch_bounds__(256)
k_splat64(SplatArgs A)
{
    __shared__ int lst[SP_CHUNK];
    __shared__ int wcnt[4];
    __shared__ double2 U[SP64_KC][SP64_T];
    __shared__ double2 Vf[SP64_KC][SP64_T];

    const int t = threadIdx.x;
    const int tx = t & 15, tz = t >> 4;
    const int tile = blockIdx.x;
    const int X0 = (tile % A.ntile1) * SP64_T, Z0 = (tile / A.ntile1) * SP64_T;
    const int split = blockIdx.y, s = blockIdx.z;
    const int64_t b0 = A.offsets[s], b1 = A.offsets[s + 1];
    const int64_t nbs = b1 - b0;
    const int64_t lo = b0 + nbs * split / A.nsplit, hi = b0 + nbs * (split + 1) / A.nsplit;
    const int64_t cap = A.cap;
    const double *F = A.f;
    const double kap1 = exp(-A.d1 * A.d1 * A.inv_eps), kap2 = exp(-A.d2 * A.d2 * A.inv_eps);

    double acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;

    for (int64_t base = lo; base < hi; base += SP_CHUNK) {
        // 1. keep the beams of this chunk whose box meets the tile
        int64_t b = base + t;
        int hit = 0;
        if (b < hi) {
            double Q1 = F[(FGA_F_STATE + 0) * cap + b], Q2 = F[(FGA_F_STATE + 1) * cap + b];
            BeamBox bx = beam_box(Q1, Q2, A.o1, A.o2, A.d1, A.d2, A.Rw1, A.Rw2, A.n1, A.n2);
            hit = (bx.lo1 <= min(bx.hi1, X0 + SP64_T - 1) && max(bx.lo1, X0) <= bx.hi1 &&
                   bx.lo2 <= min(bx.hi2, Z0 + SP64_T - 1) && max(bx.lo2, Z0) <= bx.hi2)
                      ? 1
                      : 0;
        }
        unsigned long long m = __ballot(hit);
        int lane = t & 63, wv = t >> 6;
        int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wv] = __popcll(m);
        __syncthreads();
        int wb = 0, nlist = 0;
        for (int w = 0; w < 4; ++w) {
            wb += (w < wv) ? wcnt[w] : 0;
            nlist += wcnt[w];
        }
        if (hit) lst[wb + before] = t;
        __syncthreads();

        // 2. factor batches and rank-one accumulation: 16 runs of 16 per beam
        // (8 along x1, 8 along x2), one per thread
        for (int k0 = 0; k0 < nlist; k0 += SP64_KC) {
            const int k = t >> 4;
            sp64_stage(A, k0 + k < nlist ? base + lst[k0 + k] : -1, X0, Z0, t & 15, kap1, kap2,
                       U[k], Vf[k]);
            __syncthreads();
            sp64_accumulate(U, Vf, min(SP64_KC, nlist - k0), tx, tz, acc);
            __syncthreads();
        }
    }

    double *out = A.partial + ((size_t)s * A.nsplit + split) * A.n2 * (size_t)A.n1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int i2 = Z0 + tz + 16 * j;
        if (i2 >= A.n2) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int i1 = X0 + tx + 16 * i;
            if (i1 < A.n1) out[(size_t)i2 * A.n1 + i1] = acc[i][j];
        }
    }
}

__global__ void k_zero_u32(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The splat record and the box of every beam (rec null: the boxes only)
__global__ void __launch_bounds__(256)
k_splat_prep(SplatArgs A, int nshots, SplatRec *__restrict__ rec, short4 *__restrict__ box)
{
    const int64_t nb = A.offsets[nshots];
    const int64_t cap = A.cap;
    const double inv2pe = A.inv_eps * 0.15915494309189535;
    // each workgroup takes one contiguous range of beams (so a wavefront
    // meets few shots); the loop bound is uniform over the workgroup, so
    // every lane takes part in the wavefront reductions below
    const int64_t per = ((nb + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x *
                        blockDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(nb, lo + per);
    int hold_s = -1;              // the wavefront's running shot maximum (uniform)
    unsigned hold_w = 0u;
    for (int64_t base = lo; base < hi; base += blockDim.x) {
        const int64_t b = base + threadIdx.x;
        unsigned w = 0u;          // |C a| as FP32 bits (0 for lanes past the end)
        int s = 0x7fffffff;
        if (b < hi) {
            const double *p = A.f + b;
            double Q1 = p[(FGA_F_STATE + 0) * cap], Q2 = p[(FGA_F_STATE + 1) * cap];
            double P1 = p[(FGA_F_STATE + 2) * cap], P2 = p[(FGA_F_STATE + 3) * cap];
            double S = p[(FGA_F_STATE + 4) * cap];
            double ar = p[(FGA_F_STATE + 21) * cap], ai = p[(FGA_F_STATE + 22) * cap];
            double Cr = p[4 * cap], Ci = p[5 * cap];
            BeamBox bx = beam_box(Q1, Q2, A.o1, A.o2, A.d1, A.d2, A.Rw1, A.Rw2, A.n1, A.n2);
            // W = C a as modulus and phase; the phase joins theta1
            const double Wr = Cr * ar - Ci * ai, Wi = Cr * ai + Ci * ar;
            SplatRec r;
            r.B1 = P1 * inv2pe;
            r.A1 = fma(S - P1 * Q1, inv2pe, atan2(Wi, Wr) * 0.15915494309189535);
            r.B2 = P2 * inv2pe;
            r.A2 = -P2 * Q2 * inv2pe;
            r.Q1 = Q1;
            r.Q2 = Q2;
            r.w = (float)sqrt(fma(Wr, Wr, Wi * Wi));
            r.pad = 0.f;
            // empty boxes stay empty after narrowing (lo > hi)
            r.lo1 = (short)min(bx.lo1, A.n1);
            r.hi1 = (short)max(bx.hi1, -1);
            r.lo2 = (short)min(bx.lo2, A.n2);
            r.hi2 = (short)max(bx.hi2, -1);
            if (rec) rec[b] = r;
            box[b] = make_short4(r.lo1, r.hi1, r.lo2, r.hi2);
            if (A.wmax) {
                s = (int)(A.id[b] / A.per_shot);
                w = __float_as_uint(r.w);
            }
        }
        if (A.wmax) {
            // the shot's largest |C a| (non-negative floats order like their bit
            // patterns): held per wavefront while its lanes see one shot, one
            // atomic when the shot changes; lanes of a mixed round add their own
            int slo = s, shi = s == 0x7fffffff ? -1 : s;
            unsigned wm = w;
            for (int o = 32; o > 0; o >>= 1) {
                slo = min(slo, __shfl_xor(slo, o));
                shi = max(shi, __shfl_xor(shi, o));
                wm = max(wm, (unsigned)__shfl_xor((int)wm, o));
            }
            if (slo == shi) {
                if (slo != hold_s) {
                    if (hold_s >= 0 && (threadIdx.x & 63) == 0) atomicMax(&A.wmax[hold_s], hold_w);
                    hold_s = slo;
                    hold_w = wm;
                } else {
                    hold_w = max(hold_w, wm);
                }
            } else if (slo <= shi && b < hi) {
                atomicMax(&A.wmax[s], w);
            }
        }
    }
    if (A.wmax && hold_s >= 0 && (threadIdx.x & 63) == 0) atomicMax(&A.wmax[hold_s], hold_w);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_splat_mfma(SplatArgs A, int nunits, const SplatRec *__restrict__ rec,
             const short4 *__restrict__ box)
{
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (unit >= nunits) return;   // whole wavefronts leave; no workgroup barrier below
    const int ntiles = A.ntile1 * ((A.n2 + SP_T - 1) / SP_T);
    const int tile = unit % ntiles;
    const int split = (unit / ntiles) % A.nsplit;
    const int s = unit / (ntiles * A.nsplit);
    const int X0 = (tile % A.ntile1) * SP_T, Z0 = (tile / A.ntile1) * SP_T;
    const int64_t b0 = A.offsets[s], b1 = A.offsets[s + 1];
    const int64_t nbs = b1 - b0;
    const int64_t lo = b0 + nbs * split / A.nsplit, hi = b0 + nbs * (split + 1) / A.nsplit;
    const float hl2e = (float)A.half_inv_eps * 1.4426950408889634f;
    const int i1 = X0 + lane, i2 = Z0 + lane;
    const double x1 = A.o1 + i1 * A.d1, x2 = A.o2 + i2 * A.d2;

    floatx16 acc00, acc01, acc10, acc11;
    double acc64[4][16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc00[r] = acc01[r] = acc10[r] = acc11[r] = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc64[q][r] = 0.0;
    }

    // the records of the beams of one chunk that meet the tile, compacted in
    // beam order; wavefront-private, read back with uniform addresses
    __shared__ SplatRec stage_rec[4][64];
    SplatRec *st = stage_rec[threadIdx.x >> 6];

    const short4 nobox = make_short4(1, 0, 1, 0);
    short4 bx_next = lo + lane < hi ? box[lo + lane] : nobox;
    int chunks = 0;
    for (int64_t base = lo; base < hi; base += 64) {
        const int64_t b = base + lane;
        const short4 bx = bx_next;
        // prefetch the boxes of the next chunk
        bx_next = base + 64 + lane < hi ? box[base + 64 + lane] : nobox;
        const bool hit = bx.x <= min((int)bx.y, X0 + SP_T - 1) && max((int)bx.x, X0) <= bx.y &&
                         bx.z <= min((int)bx.w, Z0 + SP_T - 1) && max((int)bx.z, Z0) <= bx.w;
        const unsigned long long mask = __ballot(hit);
        if (!mask) continue;
        const int nhit = __popcll(mask);
        if (hit) {
            const float4 *src = reinterpret_cast<const float4 *>(rec + b);
            float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
            float4 *dst = reinterpret_cast<float4 *>(st + __popcll(mask & ((1ull << lane) - 1ull)));
            dst[0] = q0;
            dst[1] = q1;
            dst[2] = q2;
            dst[3] = q3;
        }
        __builtin_amdgcn_wave_barrier();
        // software pipeline: the next record is read and its factors formed
        // while the matrix cores work on the current beam
        SplatRec r = st[0];
        Frags fr = beam_frags(r, i1, i2, x1, x2, hl2e);
        for (int k = 1; k < nhit; ++k) {
            SplatRec rn = st[k];
            tile_update(fr, acc00, acc01, acc10, acc11);
            r = rn;
            fr = beam_frags(r, i1, i2, x1, x2, hl2e);
        }
        tile_update(fr, acc00, acc01, acc10, acc11);
        __builtin_amdgcn_wave_barrier();
        // fold the FP32 sums (at most 256 beams) into FP64
        if (++chunks == 4 || base + 64 >= hi) {
            chunks = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                acc64[0][k] += (double)acc00[k];
                acc64[1][k] += (double)acc01[k];
                acc64[2][k] += (double)acc10[k];
                acc64[3][k] += (double)acc11[k];
                acc00[k] = acc01[k] = acc10[k] = acc11[k] = 0.f;
            }
        }
    }
    // sums of chunks after the last fold
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc64[0][k] += (double)acc00[k];
        acc64[1][k] += (double)acc01[k];
        acc64[2][k] += (double)acc10[k];
        acc64[3][k] += (double)acc11[k];
    }

    // D[i][j] of a 32 x 32 block: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4;
    // block (a, c) covers rows x2 = Z0 + 32 a + i and columns x1 = X0 + 32 c + j
    double *out = A.partial + ((size_t)s * A.nsplit + split) * A.n2 * (size_t)A.n1;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            int row = Z0 + 32 * (q >> 1) + 8 * (k >> 2) + 4 * (lane >> 5) + (k & 3);
            int col = X0 + 32 * (q & 1) + (lane & 31);
            if (row < A.n2 && col < A.n1) out[(size_t)row * A.n1 + col] = acc64[q][k];
        }
}

__global__ void k_splat_reduce(const double *__restrict__ partial, double *__restrict__ u,
                               int nsplit, int64_t npts, int nshots)
{
    int64_t total = npts * nshots;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t s = i / npts, x = i - s * npts;
        const double *p = partial + (size_t)s * nsplit * npts + x;
        double v = 0.0;
        for (int k = 0; k < nsplit; ++k) v += p[(size_t)k * npts];
        u[i] = v;
    }
}

bool fga_splat_binned_fits(const fga_ctx *ctx, int nshots, int T);
fga_status fga_launch_splat_binned(fga_ctx *ctx, const fga_beams *beams, int nshots, double *u,
                                   SplatArgs A, const void *rec, const void *box, int T);

fga_status fga_launch_reconstruct(fga_ctx *ctx, const fga_beams *beams, int nshots, double *u)
{
    const fga_grid &g = ctx->g;
    int nt1 = (g.n1 + SP_T - 1) / SP_T, nt2 = (g.n2 + SP_T - 1) / SP_T;
    int tiles = nt1 * nt2;
    bool mfma = ctx->prec != FGA_FP64;
    SplatArgs A{};
    A.f = beams->f;
    A.offsets = beams->offsets;
    A.cap = beams->capacity;
    A.n1 = g.n1;
    A.n2 = g.n2;
    A.o1 = g.o1;
    A.o2 = g.o2;
    A.d1 = g.d1;
    A.d2 = g.d2;
    A.eps = ctx->p.eps;
    A.inv_eps = 1.0 / ctx->p.eps;
    A.half_inv_eps = 0.5 / ctx->p.eps;
    A.Rw1 = ctx->Rw1;
    A.Rw2 = ctx->Rw2;
    A.ntile1 = nt1;
    fga_status rc;
    if (mfma) {
        rc = fga_ensure(ctx, &ctx->srec, &ctx->srec_bytes,
                        (size_t)beams->capacity * sizeof(SplatRec), "splat records");
        if (rc != FGA_OK) return rc;
        rc = fga_ensure(ctx, &ctx->sbox, &ctx->sbox_bytes,
                        (size_t)beams->capacity * sizeof(short4), "splat boxes");
        if (rc != FGA_OK) return rc;
        // FP16 split products: the record pass also gathers each shot's
        // largest |C a| for the binned splat's scaling
        const bool binned = fga_splat_binned_fits(ctx, nshots, SP_T);
        if (binned && ctx->prec == FGA_MIXED_SPLIT) {
            A.id = beams->id;
            A.per_shot = 2LL * ctx->p.nq1 * ctx->p.nq2 * ctx->p.np1 * ctx->p.np2;
            A.wmax = ctx->wmax;
            hipLaunchKernelGGL(k_zero_u32, dim3((nshots + 255) / 256), dim3(256), 0, ctx->stream,
                               ctx->wmax, nshots);
        }
        hipLaunchKernelGGL(k_splat_prep, dim3(2 * ctx->num_cu), dim3(256), 0, ctx->stream, A,
                           nshots, (SplatRec *)ctx->srec, (short4 *)ctx->sbox);
        // beams binned per tile and split into equal work items, unless the
        // tile count exceeds the binning's LDS counters
        if (binned)
            return fga_launch_splat_binned(ctx, beams, nshots, u, A, ctx->srec, ctx->sbox, SP_T);
    } else if (fga_splat_binned_fits(ctx, nshots, SP64_T)) {
        // FP64: the beams binned per 128 x 128 tile (the boxes only)
        rc = fga_ensure(ctx, &ctx->sbox, &ctx->sbox_bytes,
                        (size_t)beams->capacity * sizeof(short4), "splat boxes");
        if (rc != FGA_OK) return rc;
        hipLaunchKernelGGL(k_splat_prep, dim3(2 * ctx->num_cu), dim3(256), 0, ctx->stream, A,
                           nshots, (SplatRec *)nullptr, (short4 *)ctx->sbox);
        return fga_launch_splat_binned(ctx, beams, nshots, u, A, nullptr, ctx->sbox, SP64_T);
    }
    // every tile scans a slice of its shot's beams: enough slices for about
    // per_cu work units per CU (mixed: one wavefront per unit, so that the
    // dispatcher evens out tiles of very different load; FP64: one workgroup
    // of four wavefronts per unit, on 128 x 128 tiles)
    if (!mfma) {
        nt1 = (g.n1 + SP64_T - 1) / SP64_T;
        nt2 = (g.n2 + SP64_T - 1) / SP64_T;
        tiles = nt1 * nt2;
        A.ntile1 = nt1;
    }
    int per_cu = ctx->splat_units_per_cu > 0 ? ctx->splat_units_per_cu : (mfma ? 32 : 4);
    int want_units = per_cu * ctx->num_cu;
    int want = (want_units + tiles * nshots - 1) / (tiles * nshots);
    int nsplit = want < 1 ? 1 : (want > 256 ? 256 : want);
    A.nsplit = nsplit;
    size_t npts = (size_t)g.n1 * g.n2;
    rc = fga_ensure(ctx, (void **)&ctx->partial, &ctx->partial_bytes,
                    (size_t)nshots * nsplit * npts * sizeof(double), "splat partials");
    if (rc != FGA_OK) return rc;
    A.partial = ctx->partial;
    if (mfma) {
        int nunits = tiles * nsplit * nshots;
        hipLaunchKernelGGL(k_splat_mfma, dim3((nunits + 3) / 4), dim3(256), 0, ctx->stream, A,
                           nunits, (const SplatRec *)ctx->srec, (const short4 *)ctx->sbox);
    } else {
        hipLaunchKernelGGL(k_splat64, dim3(tiles, nsplit, nshots), dim3(256), 0,
                           ctx->stream, A);
    }
    hipLaunchKernelGGL(k_splat_reduce, dim3(1024), dim3(256), 0, ctx->stream, ctx->partial, u,
                       nsplit, (int64_t)npts, nshots);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

// ------------------------------------------------------------------ traces
// u at receiver nodes.  Workgroup (split, shot, receiver block), one slice of
// the shot's beams per split; the slices write partial sums that a second
// kernel adds in slice order.  Two forms, chosen on the device:
//  * receivers in general position: one thread per receiver, the slice's
//    beams staged through LDS, a direct exp and sincos per pair;
//  * receivers one run of consecutive nodes of a row (at most TR_ROW_MAX):
//    one lane per beam.  Along the row e(x) = e^{(i (S + P.r) - |r|^2/2)/eps}
//    (r = x - Q) steps from one column to the next by the factor rho, and
//    rho itself by the real e^{-d1^2 / eps}, so a beam costs one direct
//    evaluation and a complex product per column of its box.  The lanes'
//    terms at 16 columns at a time are summed over the wavefront by a fixed
//    reduce-scatter (four halving exchanges leave each lane one column's
//    sum over 16 lanes, two butterfly steps finish it; permlane swaps and
//    DPP moves, no LDS), per wavefront in LDS, and the four wavefronts in
//    order.
#define TR_BLOCK 256
#define TR_ROW_MAX 1024

// Whether the receivers are one run of consecutive nodes of a row: shape =
// {run, first column, row, run and nrec <= TR_ROW_MAX}.
__global__ void k_rec_shape(const int32_t *__restrict__ rec, int nrec, int n1, int *shape)
{
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int r0 = rec[0];
    for (int r = threadIdx.x; r < nrec; r += blockDim.x)
        if (rec[r] != r0 + r) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int ok = !bad && r0 >= 0 && r0 % n1 + nrec <= n1;
        shape[0] = ok;
        shape[1] = ok ? r0 % n1 : 0;
        shape[2] = ok ? r0 / n1 : 0;
        shape[3] = ok && nrec <= TR_ROW_MAX;
    }
}

fga_status fga_rec_shape_into(fga_ctx *ctx, const int32_t *rec, int nrec, int *shape)
{
    hipLaunchKernelGGL(k_rec_shape, dim3(1), dim3(256), 0, ctx->stream, rec, nrec, ctx->g.n1,
                       shape);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

fga_status fga_rec_shape(fga_ctx *ctx, const int32_t *rec, int nrec, const int **shape)
{
    fga_status rc = fga_ensure(ctx, &ctx->rec_shape, &ctx->rec_shape_bytes, 4 * sizeof(int),
                               "receiver layout");
    if (rc != FGA_OK) return rc;
    rc = fga_rec_shape_into(ctx, rec, nrec, (int *)ctx->rec_shape);
    *shape = (const int *)ctx->rec_shape;
    return rc;
}

// Lane exchanges without the LDS crossbar (ds_bpermute waits on it):
// v_permlane32_swap(x, y) exchanges the upper half of x with the lower half
// of y, v_permlane16_swap(x, y) the odd rows of x with the even rows of y, so
// after either the sum (min, max) of the two registers is, in every lane,
// that of x at lane l and l ^ 32 (16) for the lanes where the bit is clear
// and that of y for the others; DPP moves within a row of 16 (row_ror:8 is
// lane ^ 8; lane ^ 4 is row_ror:4 where bit 2 is clear, row_ror:12 where it
// is set) and within a quad (lane ^ 2, lane ^ 1).
template <int CTRL>
__device__ __forceinline__ unsigned dpp32(unsigned x)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp64(double x)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = dpp32<CTRL>((unsigned)u), hi = dpp32<CTRL>((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

#define DPP_ROR(n) (0x120 + (n))
#define DPP_QXOR1 0xb1   // quad_perm [1, 0, 3, 2]
#define DPP_QXOR2 0x4e   // quad_perm [2, 3, 0, 1]

template <bool HALF32>
__device__ __forceinline__ void swap64(double &x, double &y)
{
    const unsigned long long ux = (unsigned long long)__double_as_longlong(x);
    const unsigned long long uy = (unsigned long long)__double_as_longlong(y);
    const unsigned xl = (unsigned)ux, xh = (unsigned)(ux >> 32);
    const unsigned yl = (unsigned)uy, yh = (unsigned)(uy >> 32);
    auto l = HALF32 ? __builtin_amdgcn_permlane32_swap(xl, yl, false, false)
                    : __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    auto h = HALF32 ? __builtin_amdgcn_permlane32_swap(xh, yh, false, false)
                    : __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    x = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
    y = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
}

// v at lane ^ 4 (within the row; row_ror:k reads lane (i - k) mod 16)
__device__ __forceinline__ unsigned xor4_32(unsigned v, bool up)
{
    const unsigned a = dpp32<DPP_ROR(4)>(v), b = dpp32<DPP_ROR(12)>(v);
    return up ? a : b;
}

template <bool MAX>
__device__ __forceinline__ int tr_wave_reduce(int v)
{
    const int lane = threadIdx.x & 63;
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    {
        auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
        v = op((int)r[0], (int)r[1]);
    }
    {
        auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
        v = op((int)r[0], (int)r[1]);
    }
    v = op(v, (int)dpp32<DPP_ROR(8)>((unsigned)v));
    v = op(v, (int)xor4_32((unsigned)v, (lane & 4) != 0));
    v = op(v, (int)dpp32<DPP_QXOR2>((unsigned)v));
    v = op(v, (int)dpp32<DPP_QXOR1>((unsigned)v));
    return v;
}

__device__ __forceinline__ int tr_wave_min(int v) { return tr_wave_reduce<false>(v); }
__device__ __forceinline__ int tr_wave_max(int v) { return tr_wave_reduce<true>(v); }

// the row form for beams [lo, hi) of one shot: out[r] for the receiver at
// column run1 + r of row run2; acc = [4][nrec] doubles of LDS
__device__ void trace_row(const SplatArgs &A, double *acc, int run1, int run2, int nrec,
                          int64_t lo, int64_t hi, double *out)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 4 * nrec; i += TR_BLOCK) acc[i] = 0.0;
    __syncthreads();
    double *mine = acc + w * nrec;
    const int64_t cap = A.cap;
    const double x2 = A.o2 + run2 * A.d2;
    const double kap = exp(-A.d1 * A.d1 * A.inv_eps);
    for (int64_t base = lo + 64 * w; base < hi; base += 4 * 64) {
        const int64_t b = base + lane;
        int a1 = 1, b1 = 0;                       // empty column range
        double er = 0.0, ei = 0.0, rr = 0.0, ri = 0.0, Wr = 0.0, Wi = 0.0;
        if (b < hi) {
            const double *p = A.f + b;
            const double Q1 = p[(FGA_F_STATE + 0) * cap], Q2 = p[(FGA_F_STATE + 1) * cap];
            const BeamBox bx = beam_box(Q1, Q2, A.o1, A.o2, A.d1, A.d2, A.Rw1, A.Rw2, A.n1, A.n2);
            if (run2 >= bx.lo2 && run2 <= bx.hi2) {
                a1 = max(bx.lo1, run1);
                b1 = min(bx.hi1, run1 + nrec - 1);
            }
            if (a1 <= b1) {
                const double P1 = p[(FGA_F_STATE + 2) * cap], P2 = p[(FGA_F_STATE + 3) * cap];
                const double S = p[(FGA_F_STATE + 4) * cap];
                const double ar = p[(FGA_F_STATE + 21) * cap], ai = p[(FGA_F_STATE + 22) * cap];
                const double Cr = p[4 * cap], Ci = p[5 * cap];
                Wr = Cr * ar - Ci * ai;
                Wi = Cr * ai + Ci * ar;
                const double r2 = x2 - Q2, r1 = (A.o1 + a1 * A.d1) - Q1;
                double sn, cs;
                sincos((S + P1 * r1 + P2 * r2) * A.inv_eps, &sn, &cs);
                double e = exp(-(r1 * r1 + r2 * r2) * A.half_inv_eps);
                er = e * cs;
                ei = e * sn;
                sincos(P1 * A.d1 * A.inv_eps, &sn, &cs);
                e = exp(-(r1 + 0.5 * A.d1) * A.d1 * A.inv_eps);
                rr = e * cs;
                ri = e * sn;
            }
        }
        const int u0 = tr_wave_min(a1 <= b1 ? a1 : 2147483647);
        const int u1 = tr_wave_max(a1 <= b1 ? b1 : -2147483647 - 1);
        // the column this lane ends up holding in each chunk of 16
        const int jl = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                       ((lane >> 2) & 1);
        for (int c0 = u0; c0 <= u1; c0 += 16) {
            double v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                v[j] = 0.0;
                if (c0 + j >= a1 && c0 + j <= b1) {
                    v[j] = Wr * er - Wi * ei;
                    const double t = er * rr - ei * ri;
                    ei = er * ri + ei * rr;
                    er = t;
                    rr *= kap;
                    ri *= kap;
                }
            }
            // lane ^ 32, lane ^ 16: after the swap the two registers hold
            // this lane's kept column and its partner's, added as before
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                swap64<true>(v[j], v[j + 8]);
                v[j] = v[j] + v[j + 8];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                swap64<false>(v[j], v[j + 4]);
                v[j] = v[j] + v[j + 4];
            }
            {
                const bool up = (lane & 8) != 0;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double send = up ? v[j] : v[j + 2];
                    const double keep = up ? v[j + 2] : v[j];
                    v[j] = keep + dpp64<DPP_ROR(8)>(send);
                }
            }
            {
                const bool up = (lane & 4) != 0;
                const double send = up ? v[0] : v[1];
                const double keep = up ? v[1] : v[0];
                const double a = dpp64<DPP_ROR(4)>(send), b = dpp64<DPP_ROR(12)>(send);
                v[0] = keep + (up ? a : b);
            }
            double t = v[0];
            t += dpp64<DPP_QXOR2>(t);
            t += dpp64<DPP_QXOR1>(t);
            if ((lane & 3) == 0 && c0 + jl <= u1) mine[c0 + jl - run1] += t;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nrec; r += TR_BLOCK)
        out[r] = ((acc[r] + acc[nrec + r]) + acc[2 * nrec + r]) + acc[3 * nrec + r];
}

__global__ void __launch_bounds__(TR_BLOCK)
k_trace_points(SplatArgs A, const int32_t *__restrict__ rec, int nrec,
               const int *__restrict__ shape, double *partial)
{
    __shared__ double lds[4 * TR_ROW_MAX];
    const int split = blockIdx.x, s = blockIdx.y;
    const int64_t b0 = A.offsets[s], b1 = A.offsets[s + 1];
    const int64_t nbs = b1 - b0;
    const int64_t lo = b0 + nbs * split / A.nsplit, hi = b0 + nbs * (split + 1) / A.nsplit;
    if (shape[3]) {
        if (blockIdx.z == 0)
            trace_row(A, lds, shape[1], shape[2], nrec, lo, hi,
                      partial + ((size_t)s * A.nsplit + split) * nrec);
        return;
    }
    double (*sb)[TR_BLOCK] = (double (*)[TR_BLOCK])lds;
    int4 *sbox = (int4 *)(lds + 7 * TR_BLOCK);   // truncation box of each staged beam
    const int r = blockIdx.z * TR_BLOCK + threadIdx.x;
    int i1 = 0, i2 = 0;
    if (r < nrec) {
        int node = rec[r];
        i1 = node % A.n1;
        i2 = node / A.n1;
    }
    const double x1 = A.o1 + i1 * A.d1, x2 = A.o2 + i2 * A.d2;
    const int64_t cap = A.cap;
    double acc = 0.0;
    for (int64_t base = lo; base < hi; base += TR_BLOCK) {
        int64_t b = base + threadIdx.x;
        if (b < hi) {
            const double *p = A.f + b;
            double ar = p[(FGA_F_STATE + 21) * cap], ai = p[(FGA_F_STATE + 22) * cap];
            double Cr = p[4 * cap], Ci = p[5 * cap];
            sb[0][threadIdx.x] = p[(FGA_F_STATE + 0) * cap];
            sb[1][threadIdx.x] = p[(FGA_F_STATE + 1) * cap];
            sb[2][threadIdx.x] = p[(FGA_F_STATE + 2) * cap];
            sb[3][threadIdx.x] = p[(FGA_F_STATE + 3) * cap];
            sb[4][threadIdx.x] = p[(FGA_F_STATE + 4) * cap];
            sb[5][threadIdx.x] = Cr * ar - Ci * ai;
            sb[6][threadIdx.x] = Cr * ai + Ci * ar;
            const BeamBox bx = beam_box(sb[0][threadIdx.x], sb[1][threadIdx.x], A.o1, A.o2, A.d1,
                                        A.d2, A.Rw1, A.Rw2, A.n1, A.n2);
            sbox[threadIdx.x] = make_int4(bx.lo1, bx.hi1, bx.lo2, bx.hi2);
        }
        __syncthreads();
        int nb = (int)min((int64_t)TR_BLOCK, hi - base);
        if (r < nrec) {
            for (int k = 0; k < nb; ++k) {
                const int4 bx = sbox[k];
                if (i1 < bx.x || i1 > bx.y || i2 < bx.z || i2 > bx.w) continue;
                double Q1 = sb[0][k], Q2 = sb[1][k];
                double r1 = x1 - Q1, r2 = x2 - Q2;
                double th = (sb[4][k] + sb[2][k] * r1 + sb[3][k] * r2) * A.inv_eps;
                double G = -(r1 * r1 + r2 * r2) * A.half_inv_eps;
                double sn, cs;
                sincos(th, &sn, &cs);
                double e = exp(G);
                acc += e * (sb[5][k] * cs - sb[6][k] * sn);
            }
        }
        __syncthreads();
    }
    if (r < nrec) partial[((size_t)s * A.nsplit + split) * nrec + r] = acc;
}

// one wavefront per trace value: lane l adds the slices l, l + 64, ... in
// order, then a fixed butterfly over the lanes
__global__ void k_trace_reduce(const double *__restrict__ partial, int nsplit, int nrec,
                               int nshots, double *out, int64_t stride_shot)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);   // uniform in the wavefront
    const int lane = threadIdx.x & 63;
    if (i >= nrec * nshots) return;
    const int s = i / nrec, r = i % nrec;
    const double *p = partial + (size_t)s * nsplit * nrec + r;
    double v = 0.0;
    for (int k = lane; k < nsplit; k += 64) v += p[(size_t)k * nrec];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) out[(size_t)s * stride_shot + r] = v;
}

int fga_trace_splits(const fga_ctx *ctx, int nshots, int nrec)
{
    const int rblocks = (nrec + TR_BLOCK - 1) / TR_BLOCK;
    int want = (4 * ctx->num_cu + nshots * rblocks - 1) / (nshots * rblocks);
    return want < 1 ? 1 : (want > 256 ? 256 : want);
}

fga_status fga_launch_trace_points(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                   const int32_t *rec, int nrec, double *out,
                                   int64_t stride_shot, const int *shape)
{
    const int nsplit = fga_trace_splits(ctx, nshots, nrec);
    fga_status rc = fga_ensure(ctx, &ctx->trace_part, &ctx->trace_part_bytes,
                               (size_t)nshots * nsplit * nrec * sizeof(double),
                               "trace partial sums");
    if (rc != FGA_OK) return rc;
    return fga_launch_trace_points_into(ctx, beams, nshots, rec, nrec, out, stride_shot, shape,
                                        (double *)ctx->trace_part, nsplit);
}

fga_status fga_launch_trace_points_into(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                        const int32_t *rec, int nrec, double *out,
                                        int64_t stride_shot, const int *shape, double *part,
                                        int nsplit)
{
    const fga_grid &g = ctx->g;
    const int rblocks = (nrec + TR_BLOCK - 1) / TR_BLOCK;
    SplatArgs A{};
    A.f = beams->f;
    A.offsets = beams->offsets;
    A.cap = beams->capacity;
    A.n1 = g.n1;
    A.n2 = g.n2;
    A.o1 = g.o1;
    A.o2 = g.o2;
    A.d1 = g.d1;
    A.d2 = g.d2;
    A.eps = ctx->p.eps;
    A.inv_eps = 1.0 / ctx->p.eps;
    A.half_inv_eps = 0.5 / ctx->p.eps;
    A.Rw1 = ctx->Rw1;
    A.Rw2 = ctx->Rw2;
    A.nsplit = nsplit;
    hipLaunchKernelGGL(k_trace_points, dim3(nsplit, nshots, rblocks), dim3(TR_BLOCK), 0,
                       ctx->stream, A, rec, nrec, shape, part);
    hipLaunchKernelGGL(k_trace_reduce, dim3((nrec * nshots + 3) / 4), dim3(256), 0,
                       ctx->stream, (const double *)part, nsplit, nrec, nshots, out,
                       stride_shot);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}
