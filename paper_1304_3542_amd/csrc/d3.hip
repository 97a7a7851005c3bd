// The frozen Gaussian approximation in three space dimensions (FP64), for
// the 3-D acoustic wave equation u_tt = c(x)^2 Lap u.  The paper states the
// method for general d; the three steps here are those of the 2-D path with
// d = 3:
//   1. FBI of f0 (and f1) on the (q,p) mesh as three separable windowed DFT
//      passes (psi eq.), branch data u_{+-,0} = (f0 +- i eps/(c(q)|p|) f1)/2,
//      the relative threshold, C = w psi/(2 pi eps)^{9/2}, Q = q, P = p,
//      S = 0, A = I, B = -iI, a = 2^{3/2};
//   2. RK4 of the ray, dynamic ray tracing (3x3 complex A, B) and amplitude
//      equations, Z^{-1} through the cofactors of Z = A + iB;
//   3. the recons eq. over each beam's truncation box.
// Beam record: f[53][capacity] = q(3), p(3), C(re, im), state(45) with the
// state Q(3) P(3) S A[3][3](re, im) B[3][3](re, im) a(re, im).
#include <limits.h>
#include <algorithm>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "fga.h"

#define F3_NST 45
#define F3_NF 53
#define F3_FS 8
#define F3_STATUS_CAPACITY 1
#define F3_STATUS_NUMERIC 2

struct fga3_ctx {
    fga3_grid g;
    fga3_params p;
    int max_shots;
    hipStream_t stream;
    int num_cu;
    int splat_slots;       // k3_splat workgroups resident at once (all CUs)
    int R[3], W[3], Rw[3];
    double norm;
    double *c;
    bool have_c;
    double2 *E[3];
    void *T1, *T2, *Psi;
    size_t T1_bytes, T2_bytes, Psi_bytes;
    double *cq;
    unsigned long long *maxbits;
    int64_t *blk;
    size_t blk_bytes;
    void *part;            // splat partial sums [nshots][nsplit][n3][n2][n1]
    size_t part_bytes;
    int64_t *status;
    char err[512];
};

static char g3_create_err[512] = "";

static fga_status f3_fail(fga3_ctx *ctx, fga_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx ? ctx->err : g3_create_err, 512, fmt, ap);
    va_end(ap);
    return st;
}

#define F3_HIP(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return f3_fail(ctx, e_ == hipErrorOutOfMemory ? FGA_ENOMEM : FGA_EHIP, "%s: %s",    \
                           #call, hipGetErrorString(e_));                                       \
    } while (0)

static fga_status f3_ensure(fga3_ctx *ctx, void **buf, size_t *have, size_t need, const char *w)
{
    if (*have >= need && *buf) return FGA_OK;
    if (*buf) {
        F3_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(*buf);
        *buf = nullptr;
        *have = 0;
    }
    if (hipMalloc(buf, need) != hipSuccess) {
        *buf = nullptr;
        return f3_fail(ctx, FGA_ENOMEM, "hipMalloc(%zu bytes) for %s failed", need, w);
    }
    *have = need;
    return FGA_OK;
}

static int f3_halfwidth(double eps, double tau, double d)
{
    return (int)ceil(sqrt(2.0 * eps * log(1.0 / tau)) / d);
}

// ------------------------------------------------------------------ velocity
//
// Tricubic B-spline with the samples as coefficients, indices clamped to the
// grid: inside the knot cell the weights of the four knots i-1 .. i+2 are the
// cubic pieces of beta3 at the fractional offset f (and their derivatives).
struct Vel3D {
    double c, g[3], K[3][3];
};

__device__ __forceinline__ void bw(double f, double w[3][4])
{
    const double g = 1.0 - f, f2 = f * f, f3 = f2 * f;
    w[0][0] = g * g * g / 6.0;
    w[0][1] = (4.0 - 6.0 * f2 + 3.0 * f3) / 6.0;
    w[0][2] = (1.0 + 3.0 * f + 3.0 * f2 - 3.0 * f3) / 6.0;
    w[0][3] = f3 / 6.0;
    w[1][0] = -0.5 * g * g;
    w[1][1] = 1.5 * f2 - 2.0 * f;
    w[1][2] = -1.5 * f2 + f + 0.5;
    w[1][3] = 0.5 * f2;
    w[2][0] = g;
    w[2][1] = 3.0 * f - 2.0;
    w[2][2] = 1.0 - 3.0 * f;
    w[2][3] = f;
}

// the three orders of the weight of knot k (0..3 for i-1 .. i+2) at offset f
__device__ __forceinline__ void bw_k(double f, int k, double &w0, double &w1, double &w2)
{
    const double g = 1.0 - f, f2 = f * f, f3 = f2 * f;
    switch (k) {
    case 0: w0 = g * g * g / 6.0; w1 = -0.5 * g * g; w2 = g; break;
    case 1: w0 = (4.0 - 6.0 * f2 + 3.0 * f3) / 6.0; w1 = 1.5 * f2 - 2.0 * f; w2 = 3.0 * f - 2.0; break;
    case 2: w0 = (1.0 + 3.0 * f + 3.0 * f2 - 3.0 * f3) / 6.0; w1 = -1.5 * f2 + f + 0.5; w2 = 1.0 - 3.0 * f; break;
    default: w0 = f3 / 6.0; w1 = 0.5 * f2; w2 = f; break;
    }
}

__device__ void vel3_eval(const double *__restrict__ c, const fga3_grid &G, const double *x,
                          Vel3D &v)
{
    const int n[3] = {G.n1, G.n2, G.n3};
    const double o[3] = {G.o1, G.o2, G.o3}, d[3] = {G.d1, G.d2, G.d3};
    double w[2][3][4];   // axes 1, 2: orders 0..2 at the four knots
    int i0[3];
    double fz = 0.0, dz1 = 0.0, dz2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double t = (x[a] - o[a]) / d[a];
        const double fl = floor(fmin(fmax(t, -4.0), (double)n[a] + 3.0));
        i0[a] = (int)fl;
        // outside the clamped cells the spline is constant (every tap reads
        // the edge value): its derivatives vanish
        const double dscale = (fl != floor(t)) ? 0.0 : 1.0 / d[a];
        if (a < 2) {
            bw(t - floor(t), w[a]);
            for (int k = 0; k < 4; ++k) {
                w[a][1][k] *= dscale;
                w[a][2][k] *= dscale * dscale;
            }
        } else {
            fz = t - floor(t);
            dz1 = dscale;
            dz2 = dscale * dscale;
        }
    }
    double c0 = 0, g1 = 0, g2 = 0, g3 = 0, k11 = 0, k12 = 0, k13 = 0, k22 = 0, k23 = 0, k33 = 0;
#pragma unroll 1
    for (int kb = 0; kb < 4; kb += 2) {
        // the 32 taps of two knot planes, every load issued before the first
        // use (left to itself the scheduler issues them two at a time, each
        // pair waited for: ~32 memory round trips per stage at one wavefront
        // per SIMD instead of 2)
        double cvs[2][4][4];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int r3 = min(max(i0[2] - 1 + kb + j, 0), n[2] - 1);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                const int r2 = min(max(i0[1] - 1 + k2, 0), n[1] - 1);
                const double *row = c + ((size_t)r3 * n[1] + r2) * n[0];
#pragma unroll
                for (int k1 = 0; k1 < 4; ++k1)
                    cvs[j][k2][k1] = row[min(max(i0[0] - 1 + k1, 0), n[0] - 1)];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double a0, a1, a2;
            bw_k(fz, kb + j, a0, a1, a2);
            a1 *= dz1;
            a2 *= dz2;
            double s00 = 0, s10 = 0, s01 = 0, s20 = 0, s11 = 0, s02 = 0;
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
                for (int k1 = 0; k1 < 4; ++k1) {
                    const double cv = cvs[j][k2][k1];
                    t0 = fma(cv, w[0][0][k1], t0);
                    t1 = fma(cv, w[0][1][k1], t1);
                    t2 = fma(cv, w[0][2][k1], t2);
                }
                s00 = fma(t0, w[1][0][k2], s00);
                s10 = fma(t1, w[1][0][k2], s10);
                s01 = fma(t0, w[1][1][k2], s01);
                s20 = fma(t2, w[1][0][k2], s20);
                s11 = fma(t1, w[1][1][k2], s11);
                s02 = fma(t0, w[1][2][k2], s02);
            }
            c0 = fma(s00, a0, c0);
            g1 = fma(s10, a0, g1);
            g2 = fma(s01, a0, g2);
            g3 = fma(s00, a1, g3);
            k11 = fma(s20, a0, k11);
            k12 = fma(s11, a0, k12);
            k13 = fma(s10, a1, k13);
            k22 = fma(s02, a0, k22);
            k23 = fma(s01, a1, k23);
            k33 = fma(s00, a2, k33);
        }
    }
    v.c = c0;
    v.g[0] = g1;
    v.g[1] = g2;
    v.g[2] = g3;
    v.K[0][0] = k11;
    v.K[0][1] = v.K[1][0] = k12;
    v.K[0][2] = v.K[2][0] = k13;
    v.K[1][1] = k22;
    v.K[1][2] = v.K[2][1] = k23;
    v.K[2][2] = k33;
}

__global__ void k3_check_c(const double *c, int64_t n, int64_t *status)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!(c[i] > 0.0) || !isfinite(c[i]))
            atomicOr((unsigned long long *)status, F3_STATUS_NUMERIC);
}

// ------------------------------------------------------------------ step 1

// E[l][m + R] = exp(-(m d)^2/(2 eps)) exp(-i p_l m d / eps)
__global__ void k3_table(double2 *E, int np, int R, double dp, double d, double eps)
{
    const int W = 2 * R + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np * W; i += gridDim.x * blockDim.x) {
        const int l = i / W, m = i % W - R;
        const double r = m * d, pl = (l - 0.5 * (np - 1)) * dp;
        double s, co;
        sincos(-pl * r / eps, &s, &co);
        const double e = exp(-r * r / (2.0 * eps));
        E[i] = double2{e * co, e * s};
    }
}

// pass 1: T1[sf][i3][i2][j1 np1 + l1] = d1 sum_m f[sf][i3][i2][k1 + m] E1[l1][m]
__global__ void k3_pass1(const double *__restrict__ f0, const double *__restrict__ f1, int nfj,
                         fga3_grid G, int qb1, int qs1, int nq1, int np1, int R1,
                         const double2 *__restrict__ E1, int S, double2 *__restrict__ T1)
{
    const int64_t NC1 = (int64_t)nq1 * np1;
    const int64_t total = (int64_t)S * G.n3 * G.n2 * NC1;
    const int W1 = 2 * R1 + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c1 = i % NC1, row = i / NC1;   // row = (sf n3 + i3) n2 + i2
        const int64_t sf = row / ((int64_t)G.n3 * G.n2), rr = row % ((int64_t)G.n3 * G.n2);
        const int j1 = (int)(c1 / np1), l1 = (int)(c1 % np1);
        const int s = (int)(sf / nfj), fj = (int)(sf % nfj);
        const double *fr = (fj == 0 ? f0 : f1) + ((size_t)s * G.n3 * G.n2 + rr) * G.n1;
        const int k1 = qb1 + j1 * qs1;
        const double2 *e = E1 + (size_t)l1 * W1 + R1;
        double ar = 0.0, ai = 0.0;
        const int mlo = max(-R1, -k1), mhi = min(R1, G.n1 - 1 - k1);
        for (int m = mlo; m <= mhi; ++m) {
            const double v = fr[k1 + m];
            ar = fma(v, e[m].x, ar);
            ai = fma(v, e[m].y, ai);
        }
        T1[i] = double2{G.d1 * ar, G.d1 * ai};
    }
}

// pass 2: T2[sf][i3][c2][c1] = d2 sum_m T1[sf][i3][k2 + m][c1] E2[l2][m]
__global__ void k3_pass2(const double2 *__restrict__ T1, fga3_grid G, int qb2, int qs2, int nq2,
                         int np2, int R2, const double2 *__restrict__ E2, int S, int64_t NC1,
                         double2 *__restrict__ T2)
{
    const int64_t NC2 = (int64_t)nq2 * np2;
    const int64_t total = (int64_t)S * G.n3 * NC2 * NC1;
    const int W2 = 2 * R2 + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c1 = i % NC1, r = i / NC1;
        const int64_t c2 = r % NC2, plane = r / NC2;   // plane = sf n3 + i3
        const int j2 = (int)(c2 / np2), l2 = (int)(c2 % np2);
        const int k2 = qb2 + j2 * qs2;
        const double2 *e = E2 + (size_t)l2 * W2 + R2;
        const double2 *t = T1 + (size_t)plane * G.n2 * NC1 + c1;
        double ar = 0.0, ai = 0.0;
        const int mlo = max(-R2, -k2), mhi = min(R2, G.n2 - 1 - k2);
        for (int m = mlo; m <= mhi; ++m) {
            const double2 a = t[(size_t)(k2 + m) * NC1], b = e[m];
            ar = fma(a.x, b.x, fma(-a.y, b.y, ar));
            ai = fma(a.x, b.y, fma(a.y, b.x, ai));
        }
        T2[i] = double2{G.d2 * ar, G.d2 * ai};
    }
}

// pass 3: Psi[sf][c3][c2][c1] = d3 sum_m T2[sf][k3 + m][c2][c1] E3[l3][m]
__global__ void k3_pass3(const double2 *__restrict__ T2, fga3_grid G, int qb3, int qs3, int nq3,
                         int np3, int R3, const double2 *__restrict__ E3, int S, int64_t NC12,
                         double2 *__restrict__ Psi)
{
    const int64_t NC3 = (int64_t)nq3 * np3;
    const int64_t total = (int64_t)S * NC3 * NC12;
    const int W3 = 2 * R3 + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c12 = i % NC12, r = i / NC12;
        const int64_t c3 = r % NC3, sf = r / NC3;
        const int j3 = (int)(c3 / np3), l3 = (int)(c3 % np3);
        const int k3 = qb3 + j3 * qs3;
        const double2 *e = E3 + (size_t)l3 * W3 + R3;
        const double2 *t = T2 + (size_t)sf * G.n3 * NC12 + c12;
        double ar = 0.0, ai = 0.0;
        const int mlo = max(-R3, -k3), mhi = min(R3, G.n3 - 1 - k3);
        for (int m = mlo; m <= mhi; ++m) {
            const double2 a = t[(size_t)(k3 + m) * NC12], b = e[m];
            ar = fma(a.x, b.x, fma(-a.y, b.y, ar));
            ai = fma(a.x, b.y, fma(a.y, b.x, ai));
        }
        Psi[i] = double2{G.d3 * ar, G.d3 * ai};
    }
}

struct Mesh3 {
    int qb[3], qs[3], nq[3], np[3];
    double dp[3];
    int64_t NQ, NP, NC1, NC2, NC3;
};

// c(q) on the q-mesh (q flat, axis 1 fastest)
__global__ void k3_cq(const double *__restrict__ c, fga3_grid G, Mesh3 M, double *cq)
{
    for (int64_t qf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; qf < M.NQ;
         qf += (int64_t)gridDim.x * blockDim.x) {
        const int j1 = (int)(qf % M.nq[0]), j2 = (int)((qf / M.nq[0]) % M.nq[1]),
                  j3 = (int)(qf / ((int64_t)M.nq[0] * M.nq[1]));
        const double x[3] = {G.o1 + (M.qb[0] + j1 * M.qs[0]) * G.d1,
                             G.o2 + (M.qb[1] + j2 * M.qs[1]) * G.d2,
                             G.o3 + (M.qb[2] + j3 * M.qs[2]) * G.d3};
        Vel3D v;
        vel3_eval(c, G, x, v);
        cq[qf] = v.c;
    }
}

// psi_{+-} of candidate (s, branch br, qf, pf)
struct Cand3 {
    int j[3], l[3];
    double p[3], pn;
};

__device__ __forceinline__ Cand3 cand3(const Mesh3 &M, int64_t qf, int64_t pf)
{
    Cand3 k;
    k.j[0] = (int)(qf % M.nq[0]);
    k.j[1] = (int)((qf / M.nq[0]) % M.nq[1]);
    k.j[2] = (int)(qf / ((int64_t)M.nq[0] * M.nq[1]));
    k.l[0] = (int)(pf % M.np[0]);
    k.l[1] = (int)((pf / M.np[0]) % M.np[1]);
    k.l[2] = (int)(pf / ((int64_t)M.np[0] * M.np[1]));
    for (int a = 0; a < 3; ++a) k.p[a] = (k.l[a] - 0.5 * (M.np[a] - 1)) * M.dp[a];
    k.pn = sqrt(k.p[0] * k.p[0] + k.p[1] * k.p[1] + k.p[2] * k.p[2]);
    return k;
}

__device__ __forceinline__ double2 psi_branch(const double2 *__restrict__ Psi, const Mesh3 &M,
                                              const double *__restrict__ cq, int nfj, double eps,
                                              int s, int br, int64_t qf, const Cand3 &k)
{
    const int64_t c1 = (int64_t)k.j[0] * M.np[0] + k.l[0];
    const int64_t c2 = (int64_t)k.j[1] * M.np[1] + k.l[1];
    const int64_t c3 = (int64_t)k.j[2] * M.np[2] + k.l[2];
    const int64_t inner = (c3 * M.NC2 + c2) * M.NC1 + c1;
    const int64_t plane = M.NC3 * M.NC2 * M.NC1;
    const double2 a = Psi[(size_t)(s * nfj) * plane + inner];
    if (nfj == 1) return double2{0.5 * a.x, 0.5 * a.y};
    const double2 b = Psi[(size_t)(s * nfj + 1) * plane + inner];
    const double r = eps / (cq[qf] * k.pn), sg = br == 0 ? 1.0 : -1.0;
    // (psi0 +- i r psi1) / 2
    return double2{0.5 * (a.x - sg * r * b.y), 0.5 * (a.y + sg * r * b.x)};
}

__global__ void k3_branch_max(const double2 *__restrict__ Psi, Mesh3 M,
                              const double *__restrict__ cq, int nfj, double eps, int nshots,
                              unsigned long long *maxbits)
{
    __shared__ double red[256];
    const int64_t per = 2 * M.NQ * M.NP;
    for (int s = 0; s < nshots; ++s) {
        double m = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int br = (int)(i / (M.NQ * M.NP));
            const int64_t rem = i % (M.NQ * M.NP), qf = rem / M.NP, pf = rem % M.NP;
            const Cand3 k = cand3(M, qf, pf);
            const double2 v = psi_branch(Psi, M, cq, nfj, eps, s, br, qf, k);
            m = fmax(m, sqrt(v.x * v.x + v.y * v.y));
        }
        red[threadIdx.x] = m;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
            __syncthreads();
        }
        if (threadIdx.x == 0 && red[0] > 0.0)
            atomicMax(&maxbits[s], (unsigned long long)__double_as_longlong(red[0]));
        __syncthreads();
    }
}

struct Keep3 {
    const double2 *Psi;
    Mesh3 M;
    const double *cq;
    const unsigned long long *maxbits;
    int nfj, nshots;
    double eps, tau;
};

// candidate id = ((s*2 + br) NQ + qf) NP + pf: kept, and psi_{+-}
__device__ __forceinline__ bool keep3(const Keep3 &K, int64_t id, double2 &psi, Cand3 &k, int &s,
                                      int &br, int64_t &qf)
{
    const int64_t NQNP = K.M.NQ * K.M.NP;
    s = (int)(id / (2 * NQNP));
    const int64_t r = id % (2 * NQNP);
    br = (int)(r / NQNP);
    const int64_t rem = r % NQNP;
    qf = rem / K.M.NP;
    const int64_t pf = rem % K.M.NP;
    k = cand3(K.M, qf, pf);
    psi = psi_branch(K.Psi, K.M, K.cq, K.nfj, K.eps, s, br, qf, k);
    const double mag = sqrt(psi.x * psi.x + psi.y * psi.y);
    const double M = __longlong_as_double((long long)K.maxbits[s]);
    return mag > 0.0 && mag >= K.tau * M;
}

// kept count of every block of 256 consecutive candidate ids
__global__ void __launch_bounds__(256) k3_count(Keep3 K, int64_t ncand, int64_t *blk)
{
    __shared__ int wc[4];
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool kp = false;
    if (id < ncand) {
        double2 psi;
        Cand3 k;
        int s, br;
        int64_t qf;
        kp = keep3(K, id, psi, k, s, br, qf);
    }
    const unsigned long long bal = __ballot(kp);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// exclusive scan of the block counts in place, total at blk[nblk] (one block)
__global__ void __launch_bounds__(1024) k3_scan(int64_t *blk, int64_t nblk)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t lo = t * per, hi = min(nblk, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += blk[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? part[t - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t c = blk[i];
        blk[i] = run;
        run += c;
    }
    if (t == 1023) blk[nblk] = part[1023];
}

__global__ void __launch_bounds__(256) k3_scatter(Keep3 K, int64_t ncand, const int64_t *blk,
                                                  int64_t nblk, fga3_grid G, double norm,
                                                  fga_beams B, int64_t *status)
{
    __shared__ int wc[4];
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool kp = false;
    double2 psi = {0.0, 0.0};
    Cand3 k;
    int s = 0, br = 0;
    int64_t qf = 0;
    if (id < ncand) kp = keep3(K, id, psi, k, s, br, qf);
    const unsigned long long bal = __ballot(kp);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) wc[wv] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wc[w];
    const unsigned long long lower = lane == 0 ? 0ull : (bal & ((~0ull) >> (64 - lane)));
    const int64_t pos = blk[blockIdx.x] + before + __popcll(lower);
    const int64_t total = blk[nblk];
    const int64_t per = 2 * K.M.NQ * K.M.NP;
    // offsets never exceed the capacity: the later steps then stay in the
    // buffer even after an overflow (which the status reports)
    if (id < ncand && id % per == 0) B.offsets[id / per] = min(pos, B.capacity);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        B.offsets[K.nshots] = min(total, B.capacity);
        if (total > B.capacity) {
            atomicOr((unsigned long long *)&status[0], F3_STATUS_CAPACITY);
            atomicMax((unsigned long long *)&status[1], (unsigned long long)total);
        }
    }
    if (!kp || pos >= B.capacity) return;
    const int64_t cap = B.capacity;
    double *f = B.f + pos;
    const double q[3] = {G.o1 + (K.M.qb[0] + k.j[0] * K.M.qs[0]) * G.d1,
                         G.o2 + (K.M.qb[1] + k.j[1] * K.M.qs[1]) * G.d2,
                         G.o3 + (K.M.qb[2] + k.j[2] * K.M.qs[2]) * G.d3};
    for (int a = 0; a < 3; ++a) {
        f[(size_t)a * cap] = q[a];
        f[(size_t)(3 + a) * cap] = k.p[a];
        f[(size_t)(F3_FS + a) * cap] = q[a];
        f[(size_t)(F3_FS + 3 + a) * cap] = k.p[a];
    }
    f[(size_t)6 * cap] = norm * psi.x;
    f[(size_t)7 * cap] = norm * psi.y;
    f[(size_t)(F3_FS + 6) * cap] = 0.0;
    for (int i = 7; i < 43; ++i) f[(size_t)(F3_FS + i) * cap] = 0.0;
    for (int j = 0; j < 3; ++j) {
        f[(size_t)(F3_FS + 7 + 8 * j) * cap] = 1.0;     // A = I
        f[(size_t)(F3_FS + 26 + 8 * j) * cap] = -1.0;   // B = -iI
    }
    f[(size_t)(F3_FS + 43) * cap] = 2.0 * sqrt(2.0);    // a = 2^{3/2}
    f[(size_t)(F3_FS + 44) * cap] = 0.0;
    B.id[pos] = id;
}

// ------------------------------------------------------------------ step 2

struct C2 {
    double r, i;
};
__device__ __forceinline__ C2 cm(C2 a, C2 b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ C2 csb(C2 a, C2 b) { return {a.r - b.r, a.i - b.i}; }

struct St3 {
    double Q[3], P[3], S;
    C2 A[3][3], B[3][3], a;
};

__device__ void load3(const double *f, int64_t cap, St3 &y)
{
    for (int a = 0; a < 3; ++a) {
        y.Q[a] = f[(size_t)a * cap];
        y.P[a] = f[(size_t)(3 + a) * cap];
    }
    y.S = f[(size_t)6 * cap];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            y.A[j][k] = {f[(size_t)(7 + 2 * (3 * j + k)) * cap], f[(size_t)(8 + 2 * (3 * j + k)) * cap]};
            y.B[j][k] = {f[(size_t)(25 + 2 * (3 * j + k)) * cap], f[(size_t)(26 + 2 * (3 * j + k)) * cap]};
        }
    y.a = {f[(size_t)43 * cap], f[(size_t)44 * cap]};
}

__device__ void store3(double *f, int64_t cap, const St3 &y)
{
    for (int a = 0; a < 3; ++a) {
        f[(size_t)a * cap] = y.Q[a];
        f[(size_t)(3 + a) * cap] = y.P[a];
    }
    f[(size_t)6 * cap] = y.S;
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            f[(size_t)(7 + 2 * (3 * j + k)) * cap] = y.A[j][k].r;
            f[(size_t)(8 + 2 * (3 * j + k)) * cap] = y.A[j][k].i;
            f[(size_t)(25 + 2 * (3 * j + k)) * cap] = y.B[j][k].r;
            f[(size_t)(26 + 2 * (3 * j + k)) * cap] = y.B[j][k].i;
        }
    f[(size_t)43 * cap] = y.a.r;
    f[(size_t)44 * cap] = y.a.i;
}

// One RK4 stage: k = f(t) (branch + form: the caller signs the steps, since
// the slopes of branch - are exactly those of branch + negated), acc += wacc
// k, t = y + hnext k.  The cofactors of Z = A + iB of the stage input are
// formed first; each row of the dynamic ray tracing slopes is used for
// tr(adj(Z) dZ) and the updates as soon as it is known.
// y: the step-start state in LDS, component i at y[64 i] (this lane's column)
__device__ void stage3(const double *__restrict__ c, const fga3_grid &G, St3 &t, St3 &acc,
                       const double *y, double wacc, double hnext, bool last)
{
    Vel3D v;
    vel3_eval(c, G, t.Q, v);
    const double n = sqrt(t.P[0] * t.P[0] + t.P[1] * t.P[1] + t.P[2] * t.P[2]);
    const double inv_n = 1.0 / n;
    const double u[3] = {t.P[0] * inv_n, t.P[1] * inv_n, t.P[2] * inv_n};
    const double con = v.c * inv_n;
    const double ug = u[0] * v.g[0] + u[1] * v.g[1] + u[2] * v.g[2];
    {
        double kQ[3], kP[3];
        for (int a = 0; a < 3; ++a) {
            kQ[a] = v.c * u[a];
            kP[a] = -n * v.g[a];
        }
        const double kS = t.P[0] * kQ[0] + t.P[1] * kQ[1] + t.P[2] * kQ[2] - v.c * n;
        for (int a = 0; a < 3; ++a) {
            acc.Q[a] = fma(wacc, kQ[a], acc.Q[a]);
            acc.P[a] = fma(wacc, kP[a], acc.P[a]);
        }
        acc.S = fma(wacc, kS, acc.S);
        if (!last) {
            for (int a = 0; a < 3; ++a) {
                t.Q[a] = fma(hnext, kQ[a], y[64 * a]);
                t.P[a] = fma(hnext, kP[a], y[64 * (3 + a)]);
            }
            t.S = fma(hnext, kS, y[64 * 6]);
        }
    }
    C2 Z[3][3], cof[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) Z[j][k] = {t.A[j][k].r - t.B[j][k].i, t.A[j][k].i + t.B[j][k].r};
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            cof[j][k] = csb(cm(Z[j1][k1], Z[j2][k2]), cm(Z[j1][k2], Z[j2][k1]));
        }
    const C2 det = {Z[0][0].r * cof[0][0].r - Z[0][0].i * cof[0][0].i +
                        Z[0][1].r * cof[0][1].r - Z[0][1].i * cof[0][1].i +
                        Z[0][2].r * cof[0][2].r - Z[0][2].i * cof[0][2].i,
                    Z[0][0].r * cof[0][0].i + Z[0][0].i * cof[0][0].r +
                        Z[0][1].r * cof[0][1].i + Z[0][1].i * cof[0][1].r +
                        Z[0][2].r * cof[0][2].i + Z[0][2].i * cof[0][2].r};
    C2 tr = {0.0, 0.0};
    for (int j = 0; j < 3; ++j) {
        C2 Ag = {0.0, 0.0}, Bu = {0.0, 0.0}, AK[3];
        for (int l = 0; l < 3; ++l) {
            Ag.r = fma(t.A[j][l].r, v.g[l], Ag.r);
            Ag.i = fma(t.A[j][l].i, v.g[l], Ag.i);
            Bu.r = fma(t.B[j][l].r, u[l], Bu.r);
            Bu.i = fma(t.B[j][l].i, u[l], Bu.i);
        }
        for (int k = 0; k < 3; ++k) {
            AK[k] = {0.0, 0.0};
            for (int l = 0; l < 3; ++l) {
                AK[k].r = fma(t.A[j][l].r, v.K[l][k], AK[k].r);
                AK[k].i = fma(t.A[j][l].i, v.K[l][k], AK[k].i);
            }
        }
        const C2 m = {fma(-con, Bu.r, Ag.r), fma(-con, Bu.i, Ag.i)};
        C2 kA[3], kB[3];
        for (int k = 0; k < 3; ++k) {
            kA[k] = {fma(m.r, u[k], con * t.B[j][k].r), fma(m.i, u[k], con * t.B[j][k].i)};
            kB[k] = {-fma(n, AK[k].r, Bu.r * v.g[k]), -fma(n, AK[k].i, Bu.i * v.g[k])};
            const C2 dZ = {kA[k].r - kB[k].i, kA[k].i + kB[k].r};
            const C2 pr = cm(cof[j][k], dZ);
            tr.r += pr.r;
            tr.i += pr.i;
        }
        for (int k = 0; k < 3; ++k) {
            acc.A[j][k] = {fma(wacc, kA[k].r, acc.A[j][k].r), fma(wacc, kA[k].i, acc.A[j][k].i)};
            acc.B[j][k] = {fma(wacc, kB[k].r, acc.B[j][k].r), fma(wacc, kB[k].i, acc.B[j][k].i)};
            if (!last) {
                const int ia = 7 + 2 * (3 * j + k), ib = 25 + 2 * (3 * j + k);
                t.A[j][k] = {fma(hnext, kA[k].r, y[64 * ia]), fma(hnext, kA[k].i, y[64 * (ia + 1)])};
                t.B[j][k] = {fma(hnext, kB[k].r, y[64 * ib]), fma(hnext, kB[k].i, y[64 * (ib + 1)])};
            }
        }
    }
    // tr(Z^{-1} dZ) = tr / det
    const double id2 = 1.0 / (det.r * det.r + det.i * det.i);
    const C2 q = {(tr.r * det.r + tr.i * det.i) * id2, (tr.i * det.r - tr.r * det.i) * id2};
    const C2 ka = cm(t.a, C2{ug + 0.5 * q.r, 0.5 * q.i});
    acc.a = {fma(wacc, ka.r, acc.a.r), fma(wacc, ka.i, acc.a.i)};
    if (!last) t.a = {fma(hnext, ka.r, y[64 * 43]), fma(hnext, ka.i, y[64 * 44])};
}

__device__ __forceinline__ void st3_to(const St3 &x, double *y)
{
    for (int a = 0; a < 3; ++a) {
        y[64 * a] = x.Q[a];
        y[64 * (3 + a)] = x.P[a];
    }
    y[64 * 6] = x.S;
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            y[64 * (7 + 2 * (3 * j + k))] = x.A[j][k].r;
            y[64 * (8 + 2 * (3 * j + k))] = x.A[j][k].i;
            y[64 * (25 + 2 * (3 * j + k))] = x.B[j][k].r;
            y[64 * (26 + 2 * (3 * j + k))] = x.B[j][k].i;
        }
    y[64 * 43] = x.a.r;
    y[64 * 44] = x.a.i;
}

// One wavefront per workgroup; each lane owns a beam.  The stage input and
// the RK4 accumulator stay in registers, the step-start state in LDS (it is
// only read during the step).
__global__ void __launch_bounds__(64) k3_rk4(const double *__restrict__ c, fga3_grid G,
                                             fga_beams B, int nshots, int64_t NQNP, double dt,
                                             int nsteps, int64_t *status)
{
    __shared__ double ys_all[F3_NST * 64];
    double *ys = ys_all + threadIdx.x;
    const int64_t nb = B.offsets[nshots], cap = B.capacity;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        double *fs = B.f + (size_t)F3_FS * cap + b;
        St3 acc;
        load3(fs, cap, acc);
        st3_to(acc, ys);
        const double sdt = ((B.id[b] / NQNP) & 1) ? -dt : dt;
        const double h2 = 0.5 * sdt, h6 = sdt / 6.0, h3 = sdt / 3.0;
        for (int it = 0; it < nsteps; ++it) {
            St3 t = acc;
            // the four stages as a loop that is not unrolled: one copy of the
            // 3-D stage is compiled, so its temporaries are live only once
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const double wk = (k == 0 || k == 3) ? h6 : h3;
                const double hk = k < 2 ? h2 : (k == 2 ? sdt : 0.0);
                stage3(c, G, t, acc, ys, wk, hk, k == 3);
            }
            st3_to(acc, ys);
        }
        if (!isfinite(acc.Q[0]) || !isfinite(acc.a.r) || !isfinite(acc.a.i))
            atomicOr((unsigned long long *)status, F3_STATUS_NUMERIC);
        store3(fs, cap, acc);
    }
}

// ------------------------------------------------------------------ step 3
//
// A workgroup takes one tile of 16 (x1) x 32 (x2) x 32 (x3) nodes and one
// slice of a shot's beams (each shot's beams are cut into nsplit slices);
// wavefront w owns the 8 x3 planes Z0 + 8 w + t.  The sum is separable:
// with r_a = x_a - Q_a,
//   g_a(x_a) = exp(i P_a r_a / eps - r_a^2 / (2 eps)),   W = C a exp(iS/eps),
// a beam adds Re(W g1 g2 g3) inside its truncation box and nothing outside.
// The beams are staged 48 at a time (the most that one thread per beam and
// run fits in the workgroup), their factors at the tile's coordinates formed
// as five runs of 16 (x1 carrying W, two halves of x2, two halves of x3),
// zero outside the box: a direct evaluation at the run's first node in the
// box and then
//   g(x + d) = g(x) rho(x),   rho(x + d) = rho(x) exp(-d^2 / eps)
// (exact identities of the Gaussian; the products add rounding over at most
// 15 steps).  The beams whose box meets the tile are listed and taken two at
// a time; on plane t and x2 half h the update is the real product
//   u[x1][x2] += sum_k A[x1][k] B_h[k][x2],  k = (beam of the pair, re / im),
//   A = [Re H, -Im H],  B_h = [Re g2 ; Im g2] on the half,  H = W g1(x1) g3(x3_t),
// one v_mfma_f64_16x16x4f64 each (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element i of its result is D[4 i + l / 16][l % 16]).
// The matrix cores and the FP64 vector instructions share one pipe on this
// chip, so the A operand (one product and one FMA per lane) is formed once
// per plane and used by both halves.  The slices' partial sums are added in
// slice order by k3_splat_reduce.
#define T3E 16   // tile edge in x1, and the length of every factor run
#define T3Y 32   // tile edge in x2 (two runs)
#define T3Z 32   // tile edge in x3 (two runs, 8 planes per wavefront)
#define T3B 48   // beams staged per round (T3R * T3B <= 256 threads)
#define T3R 5    // factor runs per beam: x1, x2 halves, x3 halves

typedef double d3x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256, 2) k3_splat(fga_beams B, fga3_grid G, double eps, int Rw1,
                                                int Rw2, int Rw3, int nsplit,
                                                double *__restrict__ partial)
{
    // runs: 0 = x1 (times W), 1..2 = x2 halves, 3..4 = x3 halves, beam index
    // fastest (the staging lanes write consecutive slots); slot T3B stays zero
    __shared__ double2 sg[T3R][T3E][T3B + 1];
    __shared__ int smeet[T3R][T3B];
    __shared__ int slist[T3B];
    __shared__ int snmeet;
    const int nt1 = (G.n1 + T3E - 1) / T3E;
    const int X0 = (blockIdx.x % nt1) * T3E, Z0 = (blockIdx.x / nt1) * T3Z;
    const int Y0 = blockIdx.y * T3Y;
    const int split = blockIdx.z % nsplit, s = blockIdx.z / nsplit;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t cap = B.capacity;
    const int64_t b0 = B.offsets[s], b1 = B.offsets[s + 1], nbs = b1 - b0;
    const int64_t lo = b0 + nbs * split / nsplit, hi = b0 + nbs * (split + 1) / nsplit;
    const double ieps = 1.0 / eps, hieps = 0.5 / eps;
    if (tid < T3R * T3E) sg[tid / T3E][tid % T3E][T3B] = double2{0.0, 0.0};
    // this lane's place in the products: x1 (rows of A), x2 (columns of B),
    // which beam of the pair and which part (re / im)
    const int mrow = lane % 16, kcol = lane / 16, pb = kcol / 2, part = kcol % 2;
    // wavefront w's planes 8 w .. 8 w + 7 of the tile lie in x3 run 3 + w / 2
    const int zrun = 3 + w / 2, zoff = 8 * (w % 2);
    d3x4 acc[8][2];
#pragma unroll
    for (int t = 0; t < 8; ++t)
        for (int h = 0; h < 2; ++h) acc[t][h] = d3x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = lo; c0 < hi; c0 += T3B) {
        const int nc = (int)min((int64_t)T3B, hi - c0);
        if (tid < T3R * T3B) {
            const int run = tid / T3B, bb = tid % T3B;
            const int a = run == 0 ? 0 : (run < 3 ? 1 : 2);   // axis of the run
            int m0 = 1, m1 = 0;                              // empty range
            double gr = 0.0, gi = 0.0, rr = 0.0, ri = 0.0, kap = 0.0;
            if (bb < nc) {
                const double *f = B.f + (size_t)F3_FS * cap + c0 + bb;
                const double o = a == 0 ? G.o1 : (a == 1 ? G.o2 : G.o3);
                const double d = a == 0 ? G.d1 : (a == 1 ? G.d2 : G.d3);
                const int n = a == 0 ? G.n1 : (a == 1 ? G.n2 : G.n3);
                const int Rw = a == 0 ? Rw1 : (a == 1 ? Rw2 : Rw3);
                const int t0 = a == 0 ? X0 : (a == 1 ? Y0 + (run - 1) * T3E : Z0 + (run - 3) * T3E);
                const double Q = f[(size_t)a * cap], P = f[(size_t)(3 + a) * cap];
                double t = floor((Q - o) / d + 0.5);
                t = fmin(fmax(t, -1e8), 1e8);
                const int cn = (int)t;
                const int blo = max(cn - Rw, 0), bhi = min(cn + Rw, n - 1);
                m0 = max(blo - t0, 0);
                m1 = min(bhi - t0, T3E - 1);
                if (m0 <= m1) {
                    const double r = (o + (t0 + m0) * d) - Q;
                    double sn, cs;
                    sincos(P * r * ieps, &sn, &cs);
                    double e = exp(-r * r * hieps);
                    gr = e * cs;
                    gi = e * sn;
                    if (run == 0) {
                        const double S = f[6 * cap];
                        const double Cr = B.f[(size_t)6 * cap + c0 + bb];
                        const double Ci = B.f[(size_t)7 * cap + c0 + bb];
                        const double ar = f[(size_t)43 * cap], ai = f[(size_t)44 * cap];
                        sincos(S * ieps, &sn, &cs);
                        const double wr0 = Cr * ar - Ci * ai, wi0 = Cr * ai + Ci * ar;
                        const double wr = wr0 * cs - wi0 * sn, wi = wr0 * sn + wi0 * cs;
                        const double t2 = wr * gr - wi * gi;
                        gi = wr * gi + wi * gr;
                        gr = t2;
                    }
                    sincos(P * d * ieps, &sn, &cs);
                    e = exp(-(r + 0.5 * d) * d * ieps);
                    rr = e * cs;
                    ri = e * sn;
                    kap = exp(-d * d * ieps);
                }
            }
            smeet[run][bb] = m0 <= m1;
#pragma unroll
            for (int m = 0; m < T3E; ++m) {
                if (m < m0 || m > m1) {
                    sg[run][m][bb] = double2{0.0, 0.0};
                } else {
                    sg[run][m][bb] = double2{gr, gi};
                    const double t2 = gr * rr - gi * ri;
                    gi = gr * ri + gi * rr;
                    gr = t2;
                    rr *= kap;
                    ri *= kap;
                }
            }
        }
        __syncthreads();
        // list the beams whose box meets the tile, in order
        if (w == 0) {
            const int j = lane < T3B ? lane : 0;
            const int fl = lane < T3B && smeet[0][j] && (smeet[1][j] || smeet[2][j]) &&
                           (smeet[3][j] || smeet[4][j]);
            const unsigned long long mk = __ballot(fl);
            if (fl) slist[__popcll(mk & ((1ull << lane) - 1ull))] = lane;
            if (lane == 0) snmeet = __popcll(mk);
        }
        __syncthreads();
        const int nm = snmeet;
        for (int p = 0; p < nm; p += 2) {
            const int bb = pb == 0 ? slist[p] : (p + 1 < nm ? slist[p + 1] : T3B);
            const double2 g1 = sg[0][mrow][bb];
            const double2 g2a = sg[1][mrow][bb], g2b = sg[2][mrow][bb];
            const double bva = part == 0 ? g2a.x : g2a.y, bvb = part == 0 ? g2b.x : g2b.y;
            // A = Re(g1 h) (part 0) or -Im(g1 h) (part 1), both as ca h.x + cb h.y
            const double ca = part == 0 ? g1.x : -g1.y;
            const double cb = part == 0 ? -g1.y : -g1.x;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double2 h = sg[zrun][zoff + t][bb];
                const double av = fma(ca, h.x, cb * h.y);
                acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bva, acc[t][0], 0, 0, 0);
                acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bvb, acc[t][1], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // element i of plane t, half h: x1 = X0 + 4 i + lane / 16, x2 = Y0 + 16 h + lane % 16
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i2 = Y0 + 16 * h + lane % 16;
        if (i2 >= G.n2) continue;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int i3 = Z0 + 8 * w + t;
            if (i3 >= G.n3) continue;
            double *pp = partial + (((size_t)(s * nsplit + split) * G.n3 + i3) * G.n2 + i2) * G.n1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int i1 = X0 + 4 * i + lane / 16;
                if (i1 < G.n1) pp[i1] = acc[t][h][i];
            }
        }
    }
}

// u[s][node] = the slices' partial sums added in slice order
__global__ void k3_splat_reduce(const double *__restrict__ partial, int nsplit, int nshots,
                                int64_t npts, double *__restrict__ u)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nshots * npts;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / npts, k = i - s * npts;
        const double *p = partial + (size_t)s * nsplit * npts + k;
        double v = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) v += p[(size_t)sp * npts];
        u[i] = v;
    }
}

// ------------------------------------------------------------------ C ABI

static fga_status f3_check(fga3_ctx *ctx, const fga3_grid *g, const fga3_params *p)
{
    const int n[3] = {g->n1, g->n2, g->n3};
    const double d[3] = {g->d1, g->d2, g->d3};
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 4) return f3_fail(ctx, FGA_EINVAL, "grid needs at least 4 nodes per axis");
        if (!(d[a] > 0) || !isfinite(d[a])) return f3_fail(ctx, FGA_EINVAL, "grid spacing must be positive");
        if (p->nq[a] < 1 || p->qs[a] < 1 || p->qb[a] < 0 ||
            p->qb[a] + (int64_t)(p->nq[a] - 1) * p->qs[a] >= n[a])
            return f3_fail(ctx, FGA_EINVAL, "q-mesh leaves the grid along axis %d", a + 1);
        if (p->np[a] < 2 || (p->np[a] & 1) || p->np[a] > 1024)
            return f3_fail(ctx, FGA_EINVAL, "p-mesh sizes must be even, in [2, 1024]");
        if (!(p->dp[a] > 0)) return f3_fail(ctx, FGA_EINVAL, "p-mesh spacing must be positive");
    }
    if (!(p->eps > 0) || !isfinite(p->eps)) return f3_fail(ctx, FGA_EINVAL, "eps must be positive");
    if (!(p->tau >= 0 && p->tau <= 1)) return f3_fail(ctx, FGA_EINVAL, "tau must lie in [0, 1]");
    if (!(p->tau_fbi > 0 && p->tau_fbi < 1) || !(p->tau_win > 0 && p->tau_win < 1))
        return f3_fail(ctx, FGA_EINVAL, "tau_fbi and tau_win must lie in (0, 1)");
    if (!(p->dt > 0) || !isfinite(p->dt)) return f3_fail(ctx, FGA_EINVAL, "dt must be positive");
    return FGA_OK;
}

static Mesh3 f3_mesh(const fga3_params &p)
{
    Mesh3 M;
    for (int a = 0; a < 3; ++a) {
        M.qb[a] = p.qb[a];
        M.qs[a] = p.qs[a];
        M.nq[a] = p.nq[a];
        M.np[a] = p.np[a];
        M.dp[a] = p.dp[a];
    }
    M.NQ = (int64_t)p.nq[0] * p.nq[1] * p.nq[2];
    M.NP = (int64_t)p.np[0] * p.np[1] * p.np[2];
    M.NC1 = (int64_t)p.nq[0] * p.np[0];
    M.NC2 = (int64_t)p.nq[1] * p.np[1];
    M.NC3 = (int64_t)p.nq[2] * p.np[2];
    return M;
}

extern "C" fga_status fga3_create(fga3_ctx **out, const fga3_grid *g, const fga3_params *p,
                                  int32_t max_shots, void *stream)
{
    if (!out || !g || !p) return f3_fail(nullptr, FGA_EINVAL, "null argument to fga3_create");
    *out = nullptr;
    if (max_shots < 1 || max_shots > 4096)
        return f3_fail(nullptr, FGA_EINVAL, "max_shots must lie in [1, 4096]");
    fga_status st = f3_check(nullptr, g, p);
    if (st != FGA_OK) return st;
    fga3_ctx *ctx = (fga3_ctx *)calloc(1, sizeof(fga3_ctx));
    if (!ctx) return f3_fail(nullptr, FGA_ENOMEM, "host allocation failed");
    ctx->g = *g;
    ctx->p = *p;
    ctx->max_shots = max_shots;
    ctx->stream = (hipStream_t)stream;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ctx->num_cu < 1) ctx->num_cu = 256;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k3_splat, 256, 0) != hipSuccess ||
        occ < 1) {
        (void)hipGetLastError();
        occ = 2;
    }
    ctx->splat_slots = ctx->num_cu * occ;
    const double d[3] = {g->d1, g->d2, g->d3};
    double w = 1.0;
    for (int a = 0; a < 3; ++a) {
        ctx->R[a] = f3_halfwidth(p->eps, p->tau_fbi, d[a]);
        ctx->W[a] = 2 * ctx->R[a] + 1;
        ctx->Rw[a] = f3_halfwidth(p->eps, p->tau_win, d[a]);
        w *= p->qs[a] * d[a] * p->dp[a];
    }
    ctx->norm = w / pow(2.0 * M_PI * p->eps, 4.5);
    const size_t nc = (size_t)g->n1 * g->n2 * g->n3;
    bool ok = hipMalloc(&ctx->c, nc * sizeof(double)) == hipSuccess &&
              hipMalloc(&ctx->status, 2 * sizeof(int64_t)) == hipSuccess &&
              hipMalloc(&ctx->maxbits, max_shots * sizeof(unsigned long long)) == hipSuccess;
    for (int a = 0; a < 3 && ok; ++a)
        ok = hipMalloc(&ctx->E[a], (size_t)p->np[a] * ctx->W[a] * sizeof(double2)) == hipSuccess;
    if (!ok) {
        fga3_destroy(ctx);
        return f3_fail(nullptr, FGA_ENOMEM, "device allocation failed in fga3_create");
    }
    (void)hipMemsetAsync(ctx->status, 0, 2 * sizeof(int64_t), ctx->stream);
    for (int a = 0; a < 3; ++a)
        hipLaunchKernelGGL(k3_table, dim3(64), dim3(256), 0, ctx->stream, ctx->E[a], p->np[a],
                           ctx->R[a], p->dp[a], d[a], p->eps);
    if (hipGetLastError() != hipSuccess) {
        fga3_destroy(ctx);
        return f3_fail(nullptr, FGA_EHIP, "table kernel launch failed");
    }
    *out = ctx;
    return FGA_OK;
}

extern "C" fga_status fga3_destroy(fga3_ctx *ctx)
{
    if (!ctx) return FGA_OK;
    (void)hipStreamSynchronize(ctx->stream);
    void *bufs[] = {ctx->c, ctx->status, ctx->maxbits, ctx->E[0], ctx->E[1], ctx->E[2],
                    ctx->T1, ctx->T2, ctx->Psi, ctx->cq, ctx->blk, ctx->part};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    free(ctx);
    return FGA_OK;
}

extern "C" fga_status fga3_set_velocity(fga3_ctx *ctx, const double *c)
{
    if (!ctx) return FGA_EINVAL;
    if (!c) return f3_fail(ctx, FGA_EINVAL, "c is null");
    const size_t nc = (size_t)ctx->g.n1 * ctx->g.n2 * ctx->g.n3;
    F3_HIP(ctx, hipMemcpyAsync(ctx->c, c, nc * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k3_check_c, dim3(256), dim3(256), 0, ctx->stream, ctx->c, (int64_t)nc,
                       ctx->status);
    F3_HIP(ctx, hipGetLastError());
    ctx->have_c = true;
    return FGA_OK;
}

static fga_status f3_beams(fga3_ctx *ctx, const fga_beams *b, int nshots)
{
    if (!b || !b->f || !b->id || !b->offsets || b->capacity < 1)
        return f3_fail(ctx, FGA_EINVAL, "beam buffers must be non-null with capacity >= 1");
    if (nshots < 1 || nshots > ctx->max_shots)
        return f3_fail(ctx, FGA_EINVAL, "nshots %d outside [1, %d]", nshots, ctx->max_shots);
    return FGA_OK;
}

extern "C" fga_status fga3_decompose(fga3_ctx *ctx, int32_t nshots, const double *f0,
                                     const double *f1, fga_beams *beams)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = f3_beams(ctx, beams, nshots);
    if (st != FGA_OK) return st;
    if (!f0) return f3_fail(ctx, FGA_EINVAL, "f0 is null");
    if (!ctx->have_c) return f3_fail(ctx, FGA_ESTATE, "fga3_set_velocity was not called");
    const fga3_grid &G = ctx->g;
    const fga3_params &p = ctx->p;
    const Mesh3 M = f3_mesh(p);
    const int nfj = f1 ? 2 : 1, S = nshots * nfj;
    const size_t t1 = (size_t)S * G.n3 * G.n2 * M.NC1 * sizeof(double2);
    const size_t t2 = (size_t)S * G.n3 * M.NC2 * M.NC1 * sizeof(double2);
    const size_t ps = (size_t)S * M.NC3 * M.NC2 * M.NC1 * sizeof(double2);
    const int64_t ncand = 2 * (int64_t)nshots * M.NQ * M.NP;
    const int64_t nblk = (ncand + 255) / 256;
    size_t cqb = 0;
    if ((st = f3_ensure(ctx, &ctx->T1, &ctx->T1_bytes, t1, "FBI pass-1 output")) != FGA_OK ||
        (st = f3_ensure(ctx, &ctx->T2, &ctx->T2_bytes, t2, "FBI pass-2 output")) != FGA_OK ||
        (st = f3_ensure(ctx, &ctx->Psi, &ctx->Psi_bytes, ps, "FBI output")) != FGA_OK ||
        (st = f3_ensure(ctx, (void **)&ctx->cq, &cqb, M.NQ * sizeof(double), "c(q)")) != FGA_OK ||
        (st = f3_ensure(ctx, (void **)&ctx->blk, &ctx->blk_bytes, (nblk + 1) * sizeof(int64_t),
                        "compaction counts")) != FGA_OK)
        return st;
    hipStream_t s = ctx->stream;
    const int grid = ctx->num_cu * 8;
    hipLaunchKernelGGL(k3_pass1, dim3(grid), dim3(256), 0, s, f0, f1, nfj, G, p.qb[0], p.qs[0],
                       p.nq[0], p.np[0], ctx->R[0], ctx->E[0], S, (double2 *)ctx->T1);
    hipLaunchKernelGGL(k3_pass2, dim3(grid), dim3(256), 0, s, (const double2 *)ctx->T1, G,
                       p.qb[1], p.qs[1], p.nq[1], p.np[1], ctx->R[1], ctx->E[1], S, M.NC1,
                       (double2 *)ctx->T2);
    hipLaunchKernelGGL(k3_pass3, dim3(grid), dim3(256), 0, s, (const double2 *)ctx->T2, G,
                       p.qb[2], p.qs[2], p.nq[2], p.np[2], ctx->R[2], ctx->E[2], S,
                       M.NC1 * M.NC2, (double2 *)ctx->Psi);
    hipLaunchKernelGGL(k3_cq, dim3((unsigned)((M.NQ + 255) / 256)), dim3(256), 0, s, ctx->c, G,
                       M, ctx->cq);
    F3_HIP(ctx, hipMemsetAsync(ctx->maxbits, 0, nshots * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k3_branch_max, dim3(ctx->num_cu * 4), dim3(256), 0, s,
                       (const double2 *)ctx->Psi, M, ctx->cq, nfj, p.eps, nshots, ctx->maxbits);
    Keep3 K = {(const double2 *)ctx->Psi, M, ctx->cq, ctx->maxbits, nfj, nshots, p.eps, p.tau};
    hipLaunchKernelGGL(k3_count, dim3((unsigned)nblk), dim3(256), 0, s, K, ncand, ctx->blk);
    hipLaunchKernelGGL(k3_scan, dim3(1), dim3(1024), 0, s, ctx->blk, nblk);
    hipLaunchKernelGGL(k3_scatter, dim3((unsigned)nblk), dim3(256), 0, s, K, ncand, ctx->blk,
                       nblk, G, ctx->norm, *beams, ctx->status);
    F3_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

extern "C" fga_status fga3_propagate(fga3_ctx *ctx, fga_beams *beams, int32_t nshots,
                                     int32_t nsteps)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = f3_beams(ctx, beams, nshots);
    if (st != FGA_OK) return st;
    if (nsteps < 0) return f3_fail(ctx, FGA_EINVAL, "nsteps must be >= 0");
    if (!ctx->have_c) return f3_fail(ctx, FGA_ESTATE, "fga3_set_velocity was not called");
    if (nsteps == 0) return FGA_OK;
    const Mesh3 M = f3_mesh(ctx->p);
    hipLaunchKernelGGL(k3_rk4, dim3(ctx->num_cu * 16), dim3(64), 0, ctx->stream, ctx->c, ctx->g,
                       *beams, nshots, M.NQ * M.NP, ctx->p.dt, nsteps, ctx->status);
    F3_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

extern "C" fga_status fga3_reconstruct(fga3_ctx *ctx, const fga_beams *beams, int32_t nshots,
                                       double *u)
{
    if (!ctx) return FGA_EINVAL;
    fga_status st = f3_beams(ctx, beams, nshots);
    if (st != FGA_OK) return st;
    if (!u) return f3_fail(ctx, FGA_EINVAL, "u is null");
    const fga3_grid &G = ctx->g;
    const int nt1 = (G.n1 + T3E - 1) / T3E, nt2 = (G.n2 + T3Y - 1) / T3Y;
    const int nt3 = (G.n3 + T3Z - 1) / T3Z;
    // slices per (shot, tile): the count whose workgroups fill the resident
    // slots most evenly, ceil(units n / slots) / n smallest (the time of the
    // launch in units of one whole (shot, tile)), the fewest slices on a tie
    const int64_t units = (int64_t)nt1 * nt2 * nt3 * nshots;
    const int64_t slots = std::max(1, ctx->splat_slots);
    const int nmax = (int)std::min<int64_t>(32, std::max(1, 65535 / nshots));
    int nsplit = 1;
    double best = 0.0;
    for (int n = 1; n <= nmax; ++n) {
        const double t = (double)((units * n + slots - 1) / slots) / n;
        if (n == 1 || t < best * (1.0 - 1e-12)) {
            best = t;
            nsplit = n;
        }
    }
    const int64_t npts = (int64_t)G.n1 * G.n2 * G.n3;
    st = f3_ensure(ctx, &ctx->part, &ctx->part_bytes,
                   (size_t)nshots * nsplit * npts * sizeof(double), "splat partial sums");
    if (st != FGA_OK) return st;
    dim3 grid((unsigned)(nt1 * nt3), (unsigned)nt2, (unsigned)(nsplit * nshots));
    hipLaunchKernelGGL(k3_splat, grid, dim3(256), 0, ctx->stream, *beams, G, ctx->p.eps,
                       ctx->Rw[0], ctx->Rw[1], ctx->Rw[2], nsplit, (double *)ctx->part);
    hipLaunchKernelGGL(k3_splat_reduce, dim3(ctx->num_cu * 4), dim3(256), 0, ctx->stream,
                       (const double *)ctx->part, nsplit, nshots, npts, u);
    F3_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

extern "C" fga_status fga3_sync_status(fga3_ctx *ctx, int64_t *needed)
{
    if (!ctx) return FGA_EINVAL;
    int64_t h[2] = {0, 0};
    F3_HIP(ctx, hipMemcpyAsync(h, ctx->status, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    F3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    F3_HIP(ctx, hipMemsetAsync(ctx->status, 0, 2 * sizeof(int64_t), ctx->stream));
    F3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (needed) *needed = h[1];
    if (h[0] & F3_STATUS_NUMERIC)
        return f3_fail(ctx, FGA_ENUMERIC, "non-finite value or c <= 0 met on the device");
    if (h[0] & F3_STATUS_CAPACITY)
        return f3_fail(ctx, FGA_ECAPACITY, "beam capacity exceeded: %lld beams needed",
                       (long long)h[1]);
    return FGA_OK;
}

extern "C" const char *fga3_last_error(const fga3_ctx *ctx)
{
    return ctx ? ctx->err : g3_create_err;
}
