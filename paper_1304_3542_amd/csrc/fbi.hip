// Step 1 of the FGA algorithm on gfx950: the local FBI transform as two
// separable windowed DFT contractions, the branch split, relative
// thresholding and compaction into the beam arrays.
//
// psi_j(q,p) = d1 d2 sum_{m1,m2} f_j(k+m) e^{-|m d|^2/(2 eps)} e^{-i p.(m d)/eps}
// (psi eq. rewritten as the Fourier transform of the windowed g_q, local
// fast FBI of the Initial wavefield decomposition section).  The kernel is
// a product of one-dimensional factors E_i[l][m] = e^{-(m d_i)^2/(2 eps)}
// e^{-i p_l m d_i/eps}, so
//   pass 1:  T[j1,l1](i2)      = sum_m1 E1[l1][m1] f(k1(j1)+m1, i2)
//   pass 2:  Psi[j2,l2][j1,l1] = sum_m2 E2[l2][m2] T[j1,l1](k2(j2)+m2)
// Pass 2 is a batched complex GEMM (M = np2, N = nq1*np1, K = box height).
#include <math.h>

#include "fga_internal.h"

template <typename R>
struct cplx {
    R re, im;
};

// ------------------------------------------------------------------ tables

template <typename R>
__global__ void k_tables(cplx<R> *E1t, cplx<R> *E2, int R1, int R2, int np1, int np2,
                         double dp1, double dp2, double d1, double d2, double eps)
{
    int W1 = 2 * R1 + 1, W2 = 2 * R2 + 1;
    int n_a = W1 * np1, n_b = W2 * np2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_a + n_b;
         i += gridDim.x * blockDim.x) {
        if (i < n_a) {
            int m = i / np1 - R1, l = i % np1;
            double r = m * d1;
            double p = (l - 0.5 * (np1 - 1)) * dp1;
            double s, c;
            sincos(p * r / eps, &s, &c);
            double g = exp(-r * r / (2.0 * eps));
            E1t[i].re = (R)(g * c);
            E1t[i].im = (R)(-g * s);
        } else {
            int j = i - n_a;
            int l = j / W2, m = j % W2 - R2;
            double r = m * d2;
            double p = (l - 0.5 * (np2 - 1)) * dp2;
            double s, c;
            sincos(p * r / eps, &s, &c);
            double g = exp(-r * r / (2.0 * eps));
            E2[j].re = (R)(g * c);
            E2[j].im = (R)(-g * s);
        }
    }
}

__global__ void k_cq(VelGrid V, double o1, double o2, double d1, double d2, int qb1, int qb2,
                     int qs1, int qs2, int nq1, int nq2, double *cq)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq1 * nq2) return;
    int j1 = i % nq1, j2 = i / nq1;
    double x1 = o1 + (qb1 + j1 * qs1) * d1, x2 = o2 + (qb2 + j2 * qs2) * d2;
    double cv, c1, c2, c11, c12, c22;
    vel_eval(V, x1, x2, cv, c1, c2, c11, c12, c22);
    cq[i] = cv;
}

// ------------------------------------------------------------------ pass 1
// T[sf][i2][j1*np1 + l1] = d1 * sum_m E1t[m][l1] f_sf[i2][k1(j1) + m]
// For each q column j1 this is a real x complex GEMM (M = rows i2,
// N = np1, K = box width): a workgroup computes a 64 x 64 tile of one j1 with
// the row windows and the table staged through LDS, 16 outputs per thread.
#define P1_BM 64
#define P1_BN 64
#define P1_BK 16

template <typename R>
__global__ void __launch_bounds__(256)
k_fbi_pass1(const double *f0, const double *f1, int nfj, const cplx<R> *__restrict__ E1t,
            cplx<R> *__restrict__ T, int n1, int n2, int R1, int qb1, int qs1, int nq1,
            int np1, double d1)
{
    __shared__ R As[P1_BK][P1_BM + 1];
    __shared__ cplx<R> Bs[P1_BK][P1_BN];
    const int sfj = blockIdx.z;
    const int sf = sfj / nq1, j1 = sfj % nq1;
    const int s = sf / nfj, fj = sf % nfj;
    const double *fs = (fj == 0 ? f0 : f1) + (size_t)s * n2 * n1;
    const int k1 = qb1 + j1 * qs1;
    const int mlo = max(-R1, -k1), mhi = min(R1, n1 - 1 - k1);
    const int K = mhi - mlo + 1;
    const int l0 = blockIdx.x * P1_BN, r0 = blockIdx.y * P1_BM;
    const int t = threadIdx.x;
    const int tn = t % 16, tm = t / 16;
    R accr[4][4], acci[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) accr[i][j] = acci[i][j] = 0;
    for (int kk = 0; kk < K; kk += P1_BK) {
        // row windows: P1_BM rows x P1_BK taps (16 consecutive doubles per row)
        for (int e = t; e < P1_BM * P1_BK; e += 256) {
            const int r = e / P1_BK, k = e % P1_BK;
            const int i2 = r0 + r;
            R v = 0;
            if (i2 < n2 && kk + k < K) v = (R)fs[(size_t)i2 * n1 + k1 + mlo + kk + k];
            As[k][r] = v;
        }
        // table: P1_BK taps x P1_BN wavenumbers
        for (int e = t; e < P1_BK * P1_BN; e += 256) {
            const int k = e / P1_BN, n = e % P1_BN;
            const int l = l0 + n;
            cplx<R> v{0, 0};
            if (l < np1 && kk + k < K) v = E1t[(size_t)(mlo + kk + k + R1) * np1 + l];
            Bs[k][n] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < P1_BK; ++k) {
            R a[4];
            cplx<R> b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[k][tm + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[k][tn + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    accr[i][j] += b[j].re * a[i];
                    acci[i][j] += b[j].im * a[i];
                }
        }
        __syncthreads();
    }
    const int NC = nq1 * np1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int i2 = r0 + tm + 16 * i;
        if (i2 >= n2) continue;
        cplx<R> *out = T + ((size_t)sf * n2 + i2) * NC + (size_t)j1 * np1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = l0 + tn + 16 * j;
            if (l >= np1) continue;
            out[l].re = accr[i][j] * (R)d1;
            out[l].im = acci[i][j] * (R)d1;
        }
    }
}

// ------------------------------------------------------------------ pass 2
// Psi[sf][j2][l2][c] = d2 * sum_m E2[l2][m] T[sf][k2(j2) + m][c]
#define P2_BM 32
#define P2_BN 64
#define P2_BK 16

template <typename R>
__global__ void __launch_bounds__(256)
k_fbi_pass2(const cplx<R> *__restrict__ T, const cplx<R> *__restrict__ E2,
            cplx<R> *__restrict__ Psi, int n2, int R2, int qb2, int qs2, int nq2, int np2,
            int NC, double d2)
{
    __shared__ cplx<R> As[P2_BK][P2_BM + 1];
    __shared__ cplx<R> Bs[P2_BK][P2_BN];
    int W2 = 2 * R2 + 1;
    int sfj = blockIdx.z;
    int sf = sfj / nq2, j2 = sfj % nq2;
    int k2 = qb2 + j2 * qs2;
    int mlo = max(-R2, -k2), mhi = min(R2, n2 - 1 - k2);
    int K = mhi - mlo + 1;
    int c0 = blockIdx.x * P2_BN, l0 = blockIdx.y * P2_BM;
    int t = threadIdx.x;
    int tn = t % 16, tm = t / 16;
    const cplx<R> *Tb = T + (size_t)sf * n2 * NC;
    R accr[2][4], acci[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) accr[i][j] = acci[i][j] = 0;

    for (int kk = 0; kk < K; kk += P2_BK) {
        // E2 tile: P2_BM x P2_BK
        for (int e = t; e < P2_BM * P2_BK; e += 256) {
            int mm = e / P2_BK, k = e % P2_BK;
            int l = l0 + mm, m = mlo + kk + k;
            cplx<R> v{0, 0};
            if (l < np2 && kk + k < K) v = E2[(size_t)l * W2 + m + R2];
            As[k][mm] = v;
        }
        // T tile: P2_BK x P2_BN
        for (int e = t; e < P2_BK * P2_BN; e += 256) {
            int k = e / P2_BN, n = e % P2_BN;
            int cc = c0 + n;
            cplx<R> v{0, 0};
            if (cc < NC && kk + k < K) v = Tb[(size_t)(k2 + mlo + kk + k) * NC + cc];
            Bs[k][n] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < P2_BK; ++k) {
            cplx<R> a[2], b[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[k][tm + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[k][tn + 16 * j];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    accr[i][j] += a[i].re * b[j].re - a[i].im * b[j].im;
                    acci[i][j] += a[i].re * b[j].im + a[i].im * b[j].re;
                }
        }
        __syncthreads();
    }
    cplx<R> *out = Psi + ((size_t)sf * nq2 + j2) * np2 * (size_t)NC;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        int l = l0 + tm + 16 * i;
        if (l >= np2) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int cc = c0 + tn + 16 * j;
            if (cc >= NC) continue;
            out[(size_t)l * NC + cc].re = accr[i][j] * (R)d2;
            out[(size_t)l * NC + cc].im = acci[i][j] * (R)d2;
        }
    }
}

// --------------------------------------------------- branches and threshold

struct CandGeom {
    int nq1, nq2, np1, np2, nfj;
    int64_t Nq, Np;      // nq1*nq2, np1*np2
    int64_t per_shot;    // 2*Nq*Np
    double dp1, dp2, eps;
};

// psi_{+-} = (psi0 +- i eps/(c(q)|p|) psi1)/2 for local candidate index cl
// (branch-major, then q flat, then p flat) of shot s.
template <typename R>
__device__ __forceinline__ void cand_psi(const cplx<R> *__restrict__ Psi,
                                         const double *__restrict__ cq, const CandGeom &G,
                                         int s, int64_t cl, R &re, R &im)
{
    int64_t NqNp = G.Nq * G.Np;
    int sb = (int)(cl / NqNp);
    int64_t rem = cl - sb * NqNp;
    int64_t qf = rem / G.Np, pf = rem - qf * G.Np;
    int j2 = (int)(qf / G.nq1), j1 = (int)(qf - (int64_t)j2 * G.nq1);
    int l2 = (int)(pf / G.np1), l1 = (int)(pf - (int64_t)l2 * G.np1);
    size_t NC = (size_t)G.nq1 * G.np1;
    size_t off = ((size_t)j2 * G.np2 + l2) * NC + (size_t)j1 * G.np1 + l1;
    size_t plane = (size_t)G.nq2 * G.np2 * NC;
    cplx<R> p0 = Psi[(size_t)(s * G.nfj) * plane + off];
    if (G.nfj == 1) {
        re = (R)0.5 * p0.re;
        im = (R)0.5 * p0.im;
        return;
    }
    cplx<R> p1 = Psi[(size_t)(s * G.nfj + 1) * plane + off];
    double pp1 = (l1 - 0.5 * (G.np1 - 1)) * G.dp1, pp2 = (l2 - 0.5 * (G.np2 - 1)) * G.dp2;
    R r = (R)(G.eps / (cq[qf] * sqrt(pp1 * pp1 + pp2 * pp2)));
    R sg = sb == 0 ? (R)1 : (R)-1;
    re = (R)0.5 * (p0.re - sg * r * p1.im);
    im = (R)0.5 * (p0.im + sg * r * p1.re);
}

template <typename R>
__device__ __forceinline__ R cabs_r(R re, R im)
{
    return sqrt(re * re + im * im);
}

template <typename R>
__global__ void __launch_bounds__(256)
k_branch_max(const cplx<R> *__restrict__ Psi, const double *__restrict__ cq, CandGeom G,
             unsigned long long *maxbits)
{
    __shared__ double red[4];
    int s = blockIdx.y;
    R best = 0;
    for (int64_t cl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cl < G.per_shot;
         cl += (int64_t)gridDim.x * blockDim.x) {
        R re, im;
        cand_psi(Psi, cq, G, s, cl, re, im);
        R m = cabs_r(re, im);
        best = m > best ? m : best;   // NaN never wins; NaN inputs are flagged elsewhere
    }
    double b = (double)best;
    for (int o = 32; o > 0; o >>= 1) b = fmax(b, __shfl_xor(b, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        // non-negative doubles order like their bit patterns
        atomicMax(&maxbits[s], (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

#define CMP_ITEMS 16
#define CMP_BLOCK 256
#define CMP_TILE (CMP_ITEMS * CMP_BLOCK)

template <typename R>
__device__ __forceinline__ bool keep_cand(R mag, R thr)
{
    return mag >= thr && mag > (R)0;
}

template <typename R>
__device__ __forceinline__ R threshold_of(const unsigned long long *maxbits, int s, double tau)
{
    double M = __longlong_as_double((long long)maxbits[s]);
    return (R)(tau * M);
}

// Per-block keep counts, blocks in candidate order.  A block covers
// CMP_TILE consecutive candidates in CMP_ITEMS rounds of CMP_BLOCK; in every
// round consecutive threads read consecutive candidates.
template <typename R>
__global__ void __launch_bounds__(CMP_BLOCK)
k_count(const cplx<R> *__restrict__ Psi, const double *__restrict__ cq, CandGeom G,
        const unsigned long long *maxbits, double tau, int64_t *blk, int nblk)
{
    __shared__ int red[CMP_BLOCK / 64];
    const int s = blockIdx.y;
    const R thr = threshold_of<R>(maxbits, s, tau);
    const int64_t base = (int64_t)blockIdx.x * CMP_TILE + threadIdx.x;
    int cnt = 0;
    for (int i = 0; i < CMP_ITEMS; ++i) {
        const int64_t cl = base + (int64_t)i * CMP_BLOCK;
        if (cl >= G.per_shot) break;
        R re, im;
        cand_psi(Psi, cq, G, s, cl, re, im);
        cnt += keep_cand(cabs_r(re, im), thr) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < CMP_BLOCK / 64; ++w) tot += red[w];
        blk[(size_t)s * nblk + blockIdx.x] = tot;
    }
}

// Exclusive scan of the block counts of all shots (one workgroup), shot
// offsets, and the capacity check.
__global__ void __launch_bounds__(1024)
k_scan_blocks(int64_t *blk, int64_t n, int nblk, int nshots, int64_t *offsets,
              int64_t capacity, int64_t *status)
{
    __shared__ int64_t part[1024];
    int t = threadIdx.x;
    int64_t per = (n + 1023) / 1024;
    int64_t lo = min((int64_t)t * per, n), hi = min(lo + per, n);
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += blk[i];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;   // exclusive prefix of this thread's segment
    for (int64_t i = lo; i < hi; ++i) {
        int64_t v = blk[i];
        blk[i] = run;
        run += v;
    }
    __syncthreads();
    if (t == 0) {
        int64_t total = part[1023];
        for (int s = 0; s < nshots; ++s) offsets[s] = min(blk[(size_t)s * nblk], capacity);
        offsets[nshots] = min(total, capacity);
        if (total > capacity) {
            atomicOr((unsigned long long *)&status[0], FGA_STATUS_CAPACITY);
            atomicMax((unsigned long long *)&status[1], (unsigned long long)total);
        }
    }
}

// Compaction in candidate order: per round, a wave ballot ranks the kept
// candidates inside each wavefront and the wavefront totals (LDS) order the
// wavefronts, so kept beams of one round land at consecutive positions.
template <typename R>
__global__ void __launch_bounds__(CMP_BLOCK)
k_scatter(const cplx<R> *__restrict__ Psi, const double *__restrict__ cq, CandGeom G,
          const unsigned long long *maxbits, double tau, const int64_t *blk, int nblk,
          fga_beams B, double o1, double o2, double d1, double d2, int qb1, int qb2,
          int qs1, int qs2, double norm)
{
    __shared__ int wsum[CMP_BLOCK / 64];
    const int s = blockIdx.y;
    const R thr = threshold_of<R>(maxbits, s, tau);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t cap = B.capacity;
    const int64_t NqNp = G.Nq * G.Np;
    int64_t run = blk[(size_t)s * nblk + blockIdx.x];
    for (int i = 0; i < CMP_ITEMS; ++i) {
        const int64_t cl = (int64_t)blockIdx.x * CMP_TILE + (int64_t)i * CMP_BLOCK + threadIdx.x;
        R re = 0, im = 0;
        bool keep = false;
        if (cl < G.per_shot) {
            cand_psi(Psi, cq, G, s, cl, re, im);
            keep = keep_cand(cabs_r(re, im), thr);
        }
        const unsigned long long m = __ballot(keep);
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int wbase = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < CMP_BLOCK / 64; ++w) {
            wbase += w < wv ? wsum[w] : 0;
            tot += wsum[w];
        }
        __syncthreads();
        const int64_t pos = run + wbase + __popcll(m & below);
        run += tot;
        if (keep && pos < cap) {
            const int sb = (int)(cl / NqNp);
            const int64_t rem = cl - sb * NqNp;
            const int64_t qf = rem / G.Np, pf = rem - qf * G.Np;
            const int j2 = (int)(qf / G.nq1), j1 = (int)(qf - (int64_t)j2 * G.nq1);
            const int l2 = (int)(pf / G.np1), l1 = (int)(pf - (int64_t)l2 * G.np1);
            const double q1 = o1 + (qb1 + j1 * qs1) * d1, q2 = o2 + (qb2 + j2 * qs2) * d2;
            const double p1 = (l1 - 0.5 * (G.np1 - 1)) * G.dp1;
            const double p2 = (l2 - 0.5 * (G.np2 - 1)) * G.dp2;
            double *f = B.f;
            f[0 * cap + pos] = q1;
            f[1 * cap + pos] = q2;
            f[2 * cap + pos] = p1;
            f[3 * cap + pos] = p2;
            f[4 * cap + pos] = norm * (double)re;
            f[5 * cap + pos] = norm * (double)im;
            const double init[FGA_NSTATE] = {q1, q2, p1, p2, 0.0,
                                             1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0,    // A = I
                                             0.0, -1.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0,  // B = -i I
                                             2.0, 0.0};                                 // a = 2
#pragma unroll
            for (int k = 0; k < FGA_NSTATE; ++k) f[(size_t)(FGA_F_STATE + k) * cap + pos] = init[k];
            B.id[pos] = (int64_t)s * G.per_shot + cl;
        }
    }
}

// ------------------------------------------------------------------ driver

template <typename R>
static fga_status decompose_impl(fga_ctx *ctx, int nshots, const double *f0, const double *f1,
                                 fga_beams *beams)
{
    const fga_grid &g = ctx->g;
    const fga_params &p = ctx->p;
    hipStream_t st = ctx->stream;
    int nfj = f1 ? 2 : 1;
    int S = nshots * nfj;
    ctx->last_nfj = nfj;
    ctx->last_nshots = nshots;
    if ((int64_t)S * std::max(p.nq1, p.nq2) > 65535)
        return fga_fail(ctx, FGA_EINVAL,
                        "nshots * (1 + (f1 != NULL)) * max(nq1, nq2) = %lld exceeds 65535",
                        (long long)S * std::max(p.nq1, p.nq2));
    size_t NC = (size_t)p.nq1 * p.np1;
    size_t e1 = (size_t)ctx->W1 * p.np1, e2 = (size_t)ctx->W2 * p.np2;

    fga_status rc;
    size_t have1 = ctx->E1t ? e1 * sizeof(cplx<R>) : 0, have2 = ctx->E2 ? e2 * sizeof(cplx<R>) : 0;
    bool fresh = !ctx->E1t || !ctx->E2;
    if ((rc = fga_ensure(ctx, &ctx->E1t, &have1, e1 * sizeof(cplx<R>), "FBI table 1")) != FGA_OK)
        return rc;
    if ((rc = fga_ensure(ctx, &ctx->E2, &have2, e2 * sizeof(cplx<R>), "FBI table 2")) != FGA_OK)
        return rc;
    if ((rc = fga_ensure(ctx, &ctx->T, &ctx->T_bytes, (size_t)S * g.n2 * NC * sizeof(cplx<R>),
                         "FBI pass-1 buffer")) != FGA_OK)
        return rc;
    if ((rc = fga_ensure(ctx, &ctx->Psi, &ctx->Psi_bytes,
                         (size_t)S * p.nq2 * p.np2 * NC * sizeof(cplx<R>), "FBI output")) != FGA_OK)
        return rc;
    CandGeom G;
    G.nq1 = p.nq1;
    G.nq2 = p.nq2;
    G.np1 = p.np1;
    G.np2 = p.np2;
    G.nfj = nfj;
    G.Nq = (int64_t)p.nq1 * p.nq2;
    G.Np = (int64_t)p.np1 * p.np2;
    G.per_shot = 2 * G.Nq * G.Np;
    G.dp1 = p.dp1;
    G.dp2 = p.dp2;
    G.eps = p.eps;
    int64_t nblk64 = (G.per_shot + CMP_TILE - 1) / CMP_TILE;
    if (nblk64 > 0x7fffffff) return fga_fail(ctx, FGA_EINVAL, "too many candidates per shot");
    int nblk = (int)nblk64;
    size_t blk_bytes = (size_t)nshots * nblk * sizeof(int64_t);
    size_t have_blk = ctx->blk_elems * sizeof(int64_t);
    if ((rc = fga_ensure(ctx, (void **)&ctx->blk, &have_blk, blk_bytes, "compaction counts")) !=
        FGA_OK)
        return rc;
    ctx->blk_elems = have_blk / sizeof(int64_t);

    if (fresh) {
        hipLaunchKernelGGL(k_tables<R>, dim3(512), dim3(256), 0, st, (cplx<R> *)ctx->E1t,
                           (cplx<R> *)ctx->E2, ctx->R1, ctx->R2, p.np1, p.np2, p.dp1, p.dp2,
                           g.d1, g.d2, p.eps);
        FGA_HIP(ctx, hipGetLastError());
    }
    int nq = p.nq1 * p.nq2;
    hipLaunchKernelGGL(k_cq, dim3((nq + 255) / 256), dim3(256), 0, st, fga_velgrid(ctx), g.o1,
                       g.o2, g.d1, g.d2, p.qb1, p.qb2, p.qs1, p.qs2, p.nq1, p.nq2, ctx->cq);
    dim3 g1((p.np1 + P1_BN - 1) / P1_BN, (g.n2 + P1_BM - 1) / P1_BM, S * p.nq1);
    hipLaunchKernelGGL(k_fbi_pass1<R>, g1, dim3(256), 0, st, f0, f1, nfj,
                       (const cplx<R> *)ctx->E1t, (cplx<R> *)ctx->T, g.n1, g.n2, ctx->R1, p.qb1,
                       p.qs1, p.nq1, p.np1, g.d1);
    dim3 g2((unsigned)((NC + P2_BN - 1) / P2_BN), (p.np2 + P2_BM - 1) / P2_BM, S * p.nq2);
    hipLaunchKernelGGL(k_fbi_pass2<R>, g2, dim3(256), 0, st, (const cplx<R> *)ctx->T,
                       (const cplx<R> *)ctx->E2, (cplx<R> *)ctx->Psi, g.n2, ctx->R2, p.qb2,
                       p.qs2, p.nq2, p.np2, (int)NC, g.d2);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, st, ctx->maxbits, nshots);
    int gmax = (int)std::min<int64_t>((G.per_shot + 255) / 256, 1024);
    hipLaunchKernelGGL(k_branch_max<R>, dim3(gmax, nshots), dim3(256), 0, st,
                       (const cplx<R> *)ctx->Psi, ctx->cq, G, ctx->maxbits);
    hipLaunchKernelGGL(k_count<R>, dim3(nblk, nshots), dim3(CMP_BLOCK), 0, st,
                       (const cplx<R> *)ctx->Psi, ctx->cq, G, ctx->maxbits, p.tau, ctx->blk, nblk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, ctx->blk,
                       (int64_t)nshots * nblk, nblk, nshots, beams->offsets, beams->capacity,
                       ctx->status);
    hipLaunchKernelGGL(k_scatter<R>, dim3(nblk, nshots), dim3(CMP_BLOCK), 0, st,
                       (const cplx<R> *)ctx->Psi, ctx->cq, G, ctx->maxbits, p.tau, ctx->blk, nblk,
                       *beams, g.o1, g.o2, g.d1, g.d2, p.qb1, p.qb2, p.qs1, p.qs2, ctx->norm);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

fga_status fga_launch_decompose(fga_ctx *ctx, int nshots, const double *f0, const double *f1,
                                fga_beams *beams)
{
    if (ctx->prec == FGA_FP64) return decompose_impl<double>(ctx, nshots, f0, f1, beams);
    return decompose_impl<float>(ctx, nshots, f0, f1, beams);
}
