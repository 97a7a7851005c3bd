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

#include <type_traits>

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
            int np1, double d1, unsigned *tmax)
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
    float big = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int i2 = r0 + tm + 16 * i;
        if (i2 >= n2) continue;
        cplx<R> *out = T + ((size_t)sf * n2 + i2) * NC + (size_t)j1 * np1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = l0 + tn + 16 * j;
            if (l >= np1) continue;
            const R vr = accr[i][j] * (R)d1, vi = acci[i][j] * (R)d1;
            out[l].re = vr;
            out[l].im = vi;
            big = fmaxf(big, fmaxf(fabsf((float)vr), fabsf((float)vi)));
        }
    }
    if (tmax) {
        // largest |Re T|, |Im T| of the (shot, part): one atomic per workgroup
        // (non-negative floats order like their bit patterns)
        __shared__ float red[4];
        for (int o = 32; o > 0; o >>= 1) big = fmaxf(big, __shfl_xor(big, o));
        if ((t & 63) == 0) red[t >> 6] = big;
        __syncthreads();
        if (t == 0)
            atomicMax(&tmax[sf], __float_as_uint(fmaxf(fmaxf(red[0], red[1]),
                                                       fmaxf(red[2], red[3]))));
    }
}

// |psi| in the precision of the path, with one explicit FMA so that every
// kernel that forms it (the pass-2 epilogue's maximum, the selection, the
// compaction) rounds it the same way
template <typename R>
__device__ __forceinline__ R cabs_r(R re, R im)
{
    return sqrt(fma(re, re, im * im));
}

// Largest |psi_+-| = |psi| / 2 of a workgroup's outputs (f1 = 0: both
// branches are psi0 / 2) folded into the shot's maximum: a wavefront
// butterfly, the four wavefronts through LDS, one atomicMax on the bit
// pattern (non-negative doubles order like their bit patterns).  NaN never
// wins here; k_count and k_scatter map it to key 0.
template <typename R>
__device__ __forceinline__ void fold_branch_max(R best, unsigned long long *maxbits, double *red)
{
    double b = (double)best;
    for (int o = 32; o > 0; o >>= 1) b = fmax(b, __shfl_xor(b, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
    }
}

// XCD-aware order of the pass-2 tiles: workgroups reach the eight XCDs in
// turn (workgroup P on XCD P % 8), and the tiles of every p2 block of one
// column block read the same rows of T.  Column blocks are dealt to the XCDs
// (column block cb on XCD cb % 8) and each XCD runs the p2 blocks of a column
// block one after another, so the T rows a tile reads are in that XCD's L2
// for the others.  gridDim.x = 8 nlb ceil(ncb / 8); false for the padding.
__device__ __forceinline__ bool p2_tile(int ncb, int nlb, int &cb, int &lb)
{
    const int P = blockIdx.x, xcd = P & 7, slot = P >> 3;
    lb = slot % nlb;
    cb = (slot / nlb) * 8 + xcd;
    return cb < ncb;
}

static inline unsigned p2_grid_x(int ncb, int nlb)
{
    return (unsigned)(8 * nlb * ((ncb + 7) / 8));
}

// ------------------------------------------------------------------ pass 2
// Psi[sf][j2][l2][c] = d2 * sum_m E2[l2][m] T[sf][k2(j2) + m][c], as a GEMM on the
// matrix cores (FP32 below; FP64 in k_fbi_pass2_mfma64).  With maxbits (f1 = 0,
// relative threshold) the epilogue also folds the shot's largest |psi_+-|.

// Pass 2 of the mixed path on the matrix cores.  A complex MAC over k is a
// K = 2 real product: with v_mfma_f32_32x32x2f32 lane l holds A[l % 32][l / 32]
// and B[l / 32][l % 32], so
//   Re Psi:  A = [Re E, -Im E] (rows l2, k = re/im part), B = [Re T ; Im T]
//   Im Psi:  A = [Im E,  Re E],                            B = [Re T ; Im T]
// two MFMAs per complex k and 32 x 32 block.  A workgroup of four wavefronts
// computes a 128 (l2) x 128 (c) tile of one (shot, j2); each wavefront a
// 64 x 64 quarter (2 x 2 blocks, Re and Im: eight FP32 accumulators).  The
// table and T are staged through LDS, 16 window rows at a time.
typedef float floatx16 __attribute__((ext_vector_type(16)));
#define P2M_T 128
#define P2M_K 16

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_fbi_pass2_mfma(const cplx<float> *__restrict__ T, const cplx<float> *__restrict__ E2,
                 cplx<float> *__restrict__ Psi, int n2, int R2, int qb2, int qs2, int nq2,
                 int np2, int NC, double d2, unsigned long long *maxbits)
{
    // [k][l2], rows padded: the staging threads write along k
    __shared__ float2 Es[P2M_K][P2M_T + 1];
    __shared__ float2 Ts[P2M_K][P2M_T];   // [k][c]
    int cb, lb;
    if (!p2_tile((NC + P2M_T - 1) / P2M_T, (np2 + P2M_T - 1) / P2M_T, cb, lb)) return;
    const int W2 = 2 * R2 + 1;
    const int sfj = blockIdx.z;
    const int sf = sfj / nq2, j2 = sfj % nq2;
    const int k2 = qb2 + j2 * qs2;
    const int mlo = max(-R2, -k2), mhi = min(R2, n2 - 1 - k2);
    const int K = mhi - mlo + 1;
    const int c0 = cb * P2M_T, l0 = lb * P2M_T;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    const int i = lane & 31;
    const bool hi = lane >= 32;
    const cplx<float> *Tb = T + (size_t)sf * n2 * NC;
    floatx16 accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) accr[a][b][r] = acci[a][b][r] = 0.f;
    // the table (128 rows x 16 window rows) and T (16 window rows x 128
    // columns) of the next chunk are loaded into registers before the current
    // chunk's MFMAs and stored to LDS after them
    constexpr int PER = P2M_T * P2M_K / 256;
    float2 pe[PER], pt[PER];
    auto load = [&](int kk) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            {
                const int r = e / P2M_K, k = e % P2M_K;
                const int l = l0 + r;
                pe[q] = make_float2(0.f, 0.f);
                if (l < np2 && kk + k < K) {
                    const cplx<float> x = E2[(size_t)l * W2 + mlo + kk + k + R2];
                    pe[q] = make_float2(x.re, x.im);
                }
            }
            {
                const int k = e / P2M_T, n = e % P2M_T;
                const int cc = c0 + n;
                pt[q] = make_float2(0.f, 0.f);
                if (cc < NC && kk + k < K) {
                    const cplx<float> x = Tb[(size_t)(k2 + mlo + kk + k) * NC + cc];
                    pt[q] = make_float2(x.re, x.im);
                }
            }
        }
    };
    load(0);
    for (int kk = 0; kk < K; kk += P2M_K) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            Es[e % P2M_K][e / P2M_K] = pe[q];
            Ts[e / P2M_T][e % P2M_T] = pt[q];
        }
        __syncthreads();
        if (kk + P2M_K < K) load(kk + P2M_K);
#pragma unroll 4
        for (int k = 0; k < P2M_K; ++k) {
            float ar[2], ai[2], b[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const float2 e = Es[k][wr * 64 + a * 32 + i];
                ar[a] = hi ? -e.y : e.x;
                ai[a] = hi ? e.x : e.y;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float2 x = Ts[k][wc * 64 + c * 32 + i];
                b[c] = hi ? x.y : x.x;
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    accr[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a], b[c], accr[a][c], 0, 0, 0);
                    acci[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[a], b[c], acci[a][c], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // D[i][j] of a 32 x 32 block: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4
    cplx<float> *out = Psi + ((size_t)sf * nq2 + j2) * np2 * (size_t)NC;
    const float s2 = (float)d2;
    float best = 0.f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int l = l0 + wr * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int cc = c0 + wc * 64 + c * 32 + (lane & 31);
                if (l < np2 && cc < NC) {
                    const float vr = accr[a][c][r] * s2, vi = acci[a][c][r] * s2;
                    out[(size_t)l * NC + cc].re = vr;
                    out[(size_t)l * NC + cc].im = vi;
                    const float m = cabs_r(0.5f * vr, 0.5f * vi);
                    best = m > best ? m : best;
                }
            }
    if (maxbits) {
        __shared__ double red[4];
        fold_branch_max(best, maxbits + sf, red);
    }
}

// Pass 2 of FGA_MIXED_SPLIT on the FP16 matrix cores: every FP32 operand x
// is staged in LDS as x_hi = fp16(x), x_lo = fp16(x - x_hi) (both rounded to
// nearest, x = x_hi + x_lo to about 2^-22 relative); T is first scaled by the
// power of two 2^ks that puts the (shot, part)'s largest component in
// [2^13, 2^14), so both splits stay in the FP16 range (|E| <= 1).  With
// v_mfma_f32_32x32x16_f16 lane l supplies A[l % 32][8 (l / 32) + t] and
// B[8 (l / 32) + t][l % 32] in slot t, so the lower half of the wavefront
// carries window row m and the upper half row m + 1, eight k slots each as
// four (Re, Im) pairs:
//   Re Psi:  A = (Er, -Ei)_hi x2, (Er, -Ei)_lo x2;  B = (Tr, Ti)_hi, _lo, _hi, _lo
//   Im Psi:  A = (Ei,  Er)_hi x2, (Ei,  Er)_lo x2;  the same B
// whose products add up to Re(E T) and Im(E T) exactly in FP32.  (Er, -Ei)
// flips the sign bit of the upper half; (Ei, Er) swaps the halves.  Tiles and
// staging as in k_fbi_pass2_mfma; the epilogue multiplies by d2 2^-ks.
__device__ __forceinline__ uint2 split_h2(float x, float y)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const h2 h = __builtin_convertvector((f2){x, y}, h2);
    const unsigned hi = __builtin_bit_cast(unsigned, h);
    const float hx = (float)__builtin_bit_cast(_Float16, (unsigned short)(hi & 0xffffu));
    const float hy = (float)__builtin_bit_cast(_Float16, (unsigned short)(hi >> 16));
    const h2 l = __builtin_convertvector((f2){x - hx, y - hy}, h2);
    return make_uint2(hi, __builtin_bit_cast(unsigned, l));
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_fbi_pass2_split(const cplx<float> *__restrict__ T, const cplx<float> *__restrict__ E2,
                  cplx<float> *__restrict__ Psi, int n2, int R2, int qb2, int qs2, int nq2,
                  int np2, int NC, double d2, const unsigned *__restrict__ tmax,
                  unsigned long long *maxbits)
{
    typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
    typedef unsigned uintx4 __attribute__((ext_vector_type(4)));
    // [k][l2]: (Er, Ei) hi, lo; rows padded: the staging threads write along k
    __shared__ uint2 Es[P2M_K][P2M_T + 1];
    __shared__ uint2 Ts[P2M_K][P2M_T];   // [k][c]:  (Tr, Ti) hi, lo
    int cb, lb;
    if (!p2_tile((NC + P2M_T - 1) / P2M_T, (np2 + P2M_T - 1) / P2M_T, cb, lb)) return;
    const int W2 = 2 * R2 + 1;
    const int sfj = blockIdx.z;
    const int sf = sfj / nq2, j2 = sfj % nq2;
    const int k2 = qb2 + j2 * qs2;
    const int mlo = max(-R2, -k2), mhi = min(R2, n2 - 1 - k2);
    const int K = mhi - mlo + 1;
    const int c0 = cb * P2M_T, l0 = lb * P2M_T;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    const int i = lane & 31, h = lane >> 5;
    // the (shot, part)'s power of two
    const float tm = __uint_as_float(tmax[sf]);
    int ks = 0;
    if (tm > 0.f && tm <= 3.0e38f) {
        int e;
        (void)frexpf(tm, &e);   // tm < 2^e
        ks = 14 - e;
    }
    const float tsc = ldexpf(1.f, ks);
    const cplx<float> *Tb = T + (size_t)sf * n2 * NC;
    floatx16 accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) accr[a][b][r] = acci[a][b][r] = 0.f;
    // the next chunk's table and T values are loaded into registers before
    // the current chunk's MFMAs and split into LDS after them, so the load
    // latency hides behind the matrix work
    constexpr int PER = P2M_T * P2M_K / 256;
    float2 pe[PER], pt[PER];
    auto load = [&](int kk) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            {
                const int r = e / P2M_K, k = e % P2M_K;
                const int l = l0 + r;
                pe[q] = make_float2(0.f, 0.f);
                if (l < np2 && kk + k < K) {
                    const cplx<float> x = E2[(size_t)l * W2 + mlo + kk + k + R2];
                    pe[q] = make_float2(x.re, x.im);
                }
            }
            {
                const int k = e / P2M_T, n = e % P2M_T;
                const int cc = c0 + n;
                pt[q] = make_float2(0.f, 0.f);
                if (cc < NC && kk + k < K) {
                    const cplx<float> x = Tb[(size_t)(k2 + mlo + kk + k) * NC + cc];
                    pt[q] = make_float2(x.re, x.im);
                }
            }
        }
    };
    load(0);
    for (int kk = 0; kk < K; kk += P2M_K) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            Es[e % P2M_K][e / P2M_K] = split_h2(pe[q].x, pe[q].y);
            Ts[e / P2M_T][e % P2M_T] = split_h2(pt[q].x * tsc, pt[q].y * tsc);
        }
        __syncthreads();
        if (kk + P2M_K < K) load(kk + P2M_K);
#pragma unroll 2
        for (int k = 0; k < P2M_K; k += 2) {
            halfx8 are[2], aim[2], b[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const uint2 e = Es[k + h][wr * 64 + a * 32 + i];
                const unsigned rh = e.x ^ 0x80000000u, rl = e.y ^ 0x80000000u;
                const unsigned ih = __builtin_amdgcn_alignbit(e.x, e.x, 16);
                const unsigned il = __builtin_amdgcn_alignbit(e.y, e.y, 16);
                are[a] = __builtin_bit_cast(halfx8, (uintx4){rh, rh, rl, rl});
                aim[a] = __builtin_bit_cast(halfx8, (uintx4){ih, ih, il, il});
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint2 x = Ts[k + h][wc * 64 + c * 32 + i];
                b[c] = __builtin_bit_cast(halfx8, (uintx4){x.x, x.y, x.x, x.y});
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    accr[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(are[a], b[c], accr[a][c], 0, 0, 0);
                    acci[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aim[a], b[c], acci[a][c], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    cplx<float> *out = Psi + ((size_t)sf * nq2 + j2) * np2 * (size_t)NC;
    const float s2 = (float)(d2 * ldexp(1.0, -ks));
    float best = 0.f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int l = l0 + wr * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int cc = c0 + wc * 64 + c * 32 + (lane & 31);
                if (l < np2 && cc < NC) {
                    const float vr = accr[a][c][r] * s2, vi = acci[a][c][r] * s2;
                    out[(size_t)l * NC + cc].re = vr;
                    out[(size_t)l * NC + cc].im = vi;
                    const float m = cabs_r(0.5f * vr, 0.5f * vi);
                    best = m > best ? m : best;
                }
            }
    if (maxbits) {
        __shared__ double red[4];
        fold_branch_max(best, maxbits + sf, red);
    }
}

// FP64 pass 2 on the matrix cores (v_mfma_f64_16x16x4f64), the same complex
// product as real ones with K doubled:
//   Re Psi:  A = [Re E, -Im E] (rows l2, k = re/im part), B = [Re T ; Im T]
//   Im Psi:  A = [Im E,  Re E],                            B = [Re T ; Im T]
// one MFMA covers two window rows.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] (l / 16 = 2 (window row of the pair) + part); element i
// of its result is D[4 i + l / 16][l % 16].  A workgroup of four wavefronts
// computes a 64 (l2) x 64 (c) tile of one (shot, j2), each wavefront a
// 32 x 32 quarter (2 x 2 blocks of 16 x 16, Re and Im); the table and T are
// staged through LDS, 16 window rows at a time.
typedef double doublex4 __attribute__((ext_vector_type(4)));
#define P2D_T 64
#define P2D_K 16

__global__ void __launch_bounds__(256)
k_fbi_pass2_mfma64(const cplx<double> *__restrict__ T, const cplx<double> *__restrict__ E2,
                   cplx<double> *__restrict__ Psi, int n2, int R2, int qb2, int qs2, int nq2,
                   int np2, int NC, double d2, unsigned long long *maxbits)
{
    __shared__ double2 Es[P2D_K][P2D_T];   // [k][l2]
    __shared__ double2 Ts[P2D_K][P2D_T];   // [k][c]
    const int W2 = 2 * R2 + 1;
    const int sfj = blockIdx.z;
    const int sf = sfj / nq2, j2 = sfj % nq2;
    const int k2 = qb2 + j2 * qs2;
    const int mlo = max(-R2, -k2), mhi = min(R2, n2 - 1 - k2);
    const int K = mhi - mlo + 1;
    const int c0 = blockIdx.x * P2D_T, l0 = blockIdx.y * P2D_T;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    const int i = lane & 15, q = lane >> 4;          // row / column in a block; K slot
    const int kp = q >> 1;                           // window row of the pair
    const bool im_part = (q & 1) != 0;
    const cplx<double> *Tb = T + (size_t)sf * n2 * NC;
    doublex4 accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) accr[a][b][r] = acci[a][b][r] = 0.0;
    for (int kk = 0; kk < K; kk += P2D_K) {
        for (int e = t; e < P2D_T * P2D_K; e += 256) {
            const int r = e / P2D_K, k = e % P2D_K;
            const int l = l0 + r;
            double2 v = make_double2(0.0, 0.0);
            if (l < np2 && kk + k < K) {
                const cplx<double> x = E2[(size_t)l * W2 + mlo + kk + k + R2];
                v = make_double2(x.re, x.im);
            }
            Es[k][r] = v;
        }
        for (int e = t; e < P2D_K * P2D_T; e += 256) {
            const int k = e / P2D_T, n = e % P2D_T;
            const int cc = c0 + n;
            double2 v = make_double2(0.0, 0.0);
            if (cc < NC && kk + k < K) {
                const cplx<double> x = Tb[(size_t)(k2 + mlo + kk + k) * NC + cc];
                v = make_double2(x.re, x.im);
            }
            Ts[k][n] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int k = 0; k < P2D_K; k += 2) {
            double ar[2], ai[2], b[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double2 e = Es[k + kp][wr * 32 + a * 16 + i];
                ar[a] = im_part ? -e.y : e.x;
                ai[a] = im_part ? e.x : e.y;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double2 x = Ts[k + kp][wc * 32 + c * 16 + i];
                b[c] = im_part ? x.y : x.x;
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    accr[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], b[c], accr[a][c], 0, 0, 0);
                    acci[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], b[c], acci[a][c], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    cplx<double> *out = Psi + ((size_t)sf * nq2 + j2) * np2 * (size_t)NC;
    double best = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int l = l0 + wr * 32 + a * 16 + 4 * r + q;
                const int cc = c0 + wc * 32 + c * 16 + i;
                if (l < np2 && cc < NC) {
                    const double vr = accr[a][c][r] * d2, vi = acci[a][c][r] * d2;
                    out[(size_t)l * NC + cc].re = vr;
                    out[(size_t)l * NC + cc].im = vi;
                    const double m = cabs_r(0.5 * vr, 0.5 * vi);
                    best = m > best ? m : best;
                }
            }
    if (maxbits) {
        __shared__ double red[4];
        fold_branch_max(best, maxbits + sf, red);
    }
}

// --------------------------------------------------- branches and threshold

// Exact division of 32-bit unsigned integers by an invariant divisor d >= 1
// through a multiply-high (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994, round-up method):
//   l = ceil(log2 d),  m = floor(2^32 (2^l - d) / d) + 1,
//   t = mulhi(m, n),   n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0).
struct FastDiv {
    uint32_t d, m;
    int s1, s2;
};

static FastDiv fast_div(uint32_t d)
{
    int l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    const unsigned __int128 num = ((unsigned __int128)1 << 32) * ((1ull << l) - d);
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)(num / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    const uint32_t t = __umulhi(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

struct CandGeom {
    int nq1, nq2, np1, np2, nfj;
    int64_t Nq, Np;      // nq1*nq2, np1*np2
    int64_t per_shot;    // 2*Nq*Np
    double dp1, dp2, eps;
    int small;           // Nq*Np < 2^32: candidate indices split in 32 bits
    FastDiv fNp, fnq1, fnp1;
};

// (branch, q node, p node) of the local candidate index cl of a shot
// (branch-major, then q flat, then p flat)
__device__ __forceinline__ void cand_index(const CandGeom &G, int64_t cl, int &sb, int64_t &qf,
                                           int &j1, int &j2, int &l1, int &l2)
{
    const int64_t NqNp = G.Nq * G.Np;
    if (G.small) {
        sb = cl >= NqNp ? 1 : 0;
        const uint32_t rem = (uint32_t)(cl - sb * NqNp);
        const uint32_t q = fdiv(rem, G.fNp), pf = rem - q * (uint32_t)G.Np;
        const uint32_t a2 = fdiv(q, G.fnq1), b2 = fdiv(pf, G.fnp1);
        qf = q;
        j2 = (int)a2;
        j1 = (int)(q - a2 * (uint32_t)G.nq1);
        l2 = (int)b2;
        l1 = (int)(pf - b2 * (uint32_t)G.np1);
    } else {
        sb = (int)(cl / NqNp);
        const int64_t rem = cl - sb * NqNp;
        qf = rem / G.Np;
        const int64_t pf = rem - qf * G.Np;
        j2 = (int)(qf / G.nq1);
        j1 = (int)(qf - (int64_t)j2 * G.nq1);
        l2 = (int)(pf / G.np1);
        l1 = (int)(pf - (int64_t)l2 * G.np1);
    }
}

// psi_{+-} = (psi0 +- i eps/(c(q)|p|) psi1)/2 for local candidate index cl
// (branch-major, then q flat, then p flat) of shot s.
template <typename R>
__device__ __forceinline__ void cand_psi(const cplx<R> *__restrict__ Psi,
                                         const double *__restrict__ cq, const CandGeom &G,
                                         int s, int64_t cl, R &re, R &im)
{
    int sb, j1, j2, l1, l2;
    int64_t qf;
    cand_index(G, cl, sb, qf, j1, j2, l1, l2);
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

__global__ void k_zero_u32_fbi(unsigned *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

#define CMP_ITEMS 16
#define CMP_BLOCK 256
#define CMP_TILE (CMP_ITEMS * CMP_BLOCK)

// ---------------------------------------------------------------- selection
// Every (shot, branch) keeps the candidates whose magnitude key is above
// Sel.key, plus the first Sel.ties of those whose key equals it, in
// candidate order.  The key is the bit pattern of |psi| (non-negative floats
// order like their bit patterns); NaN maps to 0, which is never kept.
struct Sel {
    unsigned long long key;
    long long ties;
    unsigned long long prefix;   // radix select: digits fixed so far
    long long rem;               // radix select: rank still to place (< 0: done)
};

__device__ __forceinline__ unsigned long long mag_key(float m)
{
    return isnan(m) ? 0ull : (unsigned long long)__float_as_uint(m);
}
__device__ __forceinline__ unsigned long long mag_key(double m)
{
    return isnan(m) ? 0ull : (unsigned long long)__double_as_longlong(m);
}

// Relative threshold: keep |psi| >= tau M and |psi| > 0, M the largest
// |psi| of the shot over both branches (thresholding paragraph), i.e.
// key >= key(tau M), and key > 0 when tau M = 0.
template <typename R>
__global__ void k_sel_threshold(const unsigned long long *maxbits, double tau, Sel *sel,
                                int nsb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsb) return;
    const double M = __longlong_as_double((long long)maxbits[i >> 1]);
    const unsigned long long kt = mag_key((R)(tau * M));
    sel[i].key = kt ? kt - 1 : 0;
    sel[i].ties = 0;
}

// N largest per branch (Numerical test section) by radix select on the key,
// eight bits per pass from the top: per pass a histogram of the next digit
// over the candidates that match the digits fixed so far, then the digit
// whose bucket holds the remaining rank.  After the last pass the key of the
// N-th largest is fixed, and rem of the candidates equal to it are still to
// take (the first rem in candidate order).  Fewer than N nonzero candidates:
// all of them are kept.
#define TOPN_BINS 256

__global__ void k_topn_init(Sel *sel, unsigned long long *hist, int nsb, long long n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nsb * TOPN_BINS;
         i += gridDim.x * blockDim.x) {
        hist[i] = 0ull;
        if (i < nsb) {
            sel[i].key = 0ull;
            sel[i].ties = 0;
            sel[i].prefix = 0ull;
            sel[i].rem = n;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256)
k_topn_hist(const cplx<R> *__restrict__ Psi, const double *__restrict__ cq, CandGeom G,
            const Sel *sel, unsigned long long *hist, int pass, int npass)
{
    __shared__ unsigned int h[TOPN_BINS];
    const int y = blockIdx.y, s = y >> 1, sb = y & 1;
    const Sel S = sel[y];
    if (S.rem < 0) return;   // uniform over the workgroup
    for (int d = threadIdx.x; d < TOPN_BINS; d += blockDim.x) h[d] = 0u;
    __syncthreads();
    const int shift = (npass - 1 - pass) * 8;
    const int64_t NqNp = G.Nq * G.Np;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < NqNp;
         c += (int64_t)gridDim.x * blockDim.x) {
        R re, im;
        cand_psi(Psi, cq, G, s, sb * NqNp + c, re, im);
        const unsigned long long key = mag_key(cabs_r(re, im));
        if (key == 0ull) continue;
        if (pass > 0 && (key >> (shift + 8)) != S.prefix) continue;
        atomicAdd(&h[(key >> shift) & (TOPN_BINS - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < TOPN_BINS; d += blockDim.x)
        if (h[d]) atomicAdd(&hist[(size_t)y * TOPN_BINS + d], (unsigned long long)h[d]);
}

__global__ void k_topn_pick(Sel *sel, unsigned long long *hist, int nsb, int pass, int npass)
{
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= nsb) return;
    Sel S = sel[y];
    unsigned long long *hh = hist + (size_t)y * TOPN_BINS;
    if (S.rem >= 0) {
        long long above = 0;
        int digit = -1;
        for (int d = TOPN_BINS - 1; d >= 0; --d) {
            const long long c = (long long)hh[d];
            if (above + c >= S.rem) {
                digit = d;
                break;
            }
            above += c;
        }
        if (digit < 0) {
            // fewer nonzero candidates than N (only possible in the first pass)
            S.key = 0ull;
            S.ties = 0;
            S.rem = -1;
        } else {
            S.prefix = (S.prefix << 8) | (unsigned long long)digit;
            S.rem -= above;
            if (pass == npass - 1) {
                S.key = S.prefix;
                S.ties = S.rem;
                S.rem = -1;
            }
        }
        sel[y] = S;
    }
    for (int d = 0; d < TOPN_BINS; ++d) hh[d] = 0ull;
}

// ---------------------------------------------------------------- compaction
// Blocks never straddle the two branches of a shot: a shot has 2 nblkb
// blocks, block bx covers the candidates sb NqNp + (bx - sb nblkb) CMP_TILE
// + [0, CMP_TILE) of branch sb = bx / nblkb, in CMP_ITEMS rounds of
// CMP_BLOCK consecutive candidates.
struct CmpBlock {
    int s, sb;
    int64_t first, end;   // candidate range (shot-local index)
};

__device__ __forceinline__ CmpBlock cmp_block(const CandGeom &G, int nblkb)
{
    CmpBlock B;
    B.s = blockIdx.y;
    B.sb = blockIdx.x / nblkb;
    const int64_t NqNp = G.Nq * G.Np;
    B.first = B.sb * NqNp + (int64_t)(blockIdx.x - B.sb * nblkb) * CMP_TILE;
    B.end = min(B.first + (int64_t)CMP_TILE, (B.sb + 1) * NqNp);
    return B;
}

// per block: kept-above-key count (gt) and equal-key count (eq).  With sym
// (f1 = 0: psi_+ = psi_- = psi0 / 2, and both branches have the same
// selection record) only the blocks of branch + run, and each writes its
// counts for the matching block of branch - too.
template <typename R>
__global__ void __launch_bounds__(CMP_BLOCK)
k_count(const cplx<R> *__restrict__ Psi, const double *__restrict__ cq, CandGeom G,
        const Sel *sel, int64_t *blk_gt, int64_t *blk_eq, int nblkb, int sym)
{
    __shared__ int red[2][CMP_BLOCK / 64];
    const CmpBlock B = cmp_block(G, nblkb);
    const unsigned long long K = sel[B.s * 2 + B.sb].key;
    int gt = 0, eq = 0;
    if (G.nfj == 1 && G.small) {
        // f1 = 0 and 32-bit candidate indices (uniform): every load of the
        // block is issued before the first key is formed
        const size_t NC = (size_t)G.nq1 * G.np1;
        const cplx<R> *P = Psi + (size_t)B.s * G.nq2 * G.np2 * NC;
        cplx<R> v[CMP_ITEMS];
#pragma unroll
        for (int i = 0; i < CMP_ITEMS; ++i) {
            // past the block's end the last candidate is read and not counted
            const int64_t cl = min(B.first + (int64_t)i * CMP_BLOCK + threadIdx.x, B.end - 1);
            int sb, j1, j2, l1, l2;
            int64_t qf;
            cand_index(G, cl, sb, qf, j1, j2, l1, l2);
            v[i] = P[((size_t)j2 * G.np2 + l2) * NC + (size_t)j1 * G.np1 + l1];
        }
#pragma unroll
        for (int i = 0; i < CMP_ITEMS; ++i) {
            const bool in = B.first + (int64_t)i * CMP_BLOCK + threadIdx.x < B.end;
            const unsigned long long key =
                in ? mag_key(cabs_r((R)0.5 * v[i].re, (R)0.5 * v[i].im)) : 0ull;
            gt += key > K ? 1 : 0;
            eq += (key == K && key != 0ull) ? 1 : 0;
        }
    } else {
        for (int i = 0; i < CMP_ITEMS; ++i) {
            const int64_t cl = B.first + (int64_t)i * CMP_BLOCK + threadIdx.x;
            if (cl >= B.end) break;
            R re, im;
            cand_psi(Psi, cq, G, B.s, cl, re, im);
            const unsigned long long key = mag_key(cabs_r(re, im));
            gt += key > K ? 1 : 0;
            eq += (key == K && key != 0ull) ? 1 : 0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        gt += __shfl_xor(gt, o);
        eq += __shfl_xor(eq, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = gt;
        red[1][threadIdx.x >> 6] = eq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tg = 0, te = 0;
        for (int w = 0; w < CMP_BLOCK / 64; ++w) {
            tg += red[0][w];
            te += red[1][w];
        }
        const size_t at = (size_t)B.s * 2 * nblkb + blockIdx.x;
        blk_gt[at] = tg;
        blk_eq[at] = te;
        if (sym) {
            blk_gt[at + nblkb] = tg;
            blk_eq[at + nblkb] = te;
        }
    }
}

// One workgroup per (shot, branch): exclusive scan of the equal-key counts
// over the branch's blocks (the tie rank at each block's start, into blk_eq)
// and the ties each block takes, added to its kept count (blk_gt).
__global__ void __launch_bounds__(1024)
k_scan_ties(const Sel *sel, int64_t *blk_gt, int64_t *blk_eq, int nblkb)
{
    __shared__ int64_t part[1024];
    const int y = blockIdx.x;   // shot * 2 + branch
    const long long ties = sel[y].ties;
    int64_t *eq = blk_eq + (size_t)y * nblkb;
    int64_t *gt = blk_gt + (size_t)y * nblkb;
    const int t = threadIdx.x;
    const int per = (nblkb + 1023) / 1024;
    const int lo = min(t * per, nblkb), hi = min(lo + per, nblkb);
    int64_t sum = 0;
    for (int i = lo; i < hi; ++i) sum += eq[i];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int i = lo; i < hi; ++i) {
        const int64_t e = eq[i];
        const int64_t take = min(max((int64_t)ties - run, (int64_t)0), e);
        gt[i] += take;
        eq[i] = run;
        run += e;
    }
}

// Exclusive scan of the block counts of all shots, in place, in three
// launches over SCAN_SEGS contiguous segments: the segments' sums, their
// exclusive scan (one workgroup; also the total, the last shot offset and the
// capacity check), then every segment scanned from its base in tiles of 1024
// (the first blocks of the shots give the other shot offsets).
#define SCAN_SEGS 1024

// inclusive scan over the workgroup of 1024 threads; returns the inclusive
// value of this thread, total = the workgroup's sum
__device__ __forceinline__ int64_t block_scan1024(int64_t v, int64_t *wsum, int64_t &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    int64_t base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        base += w < wv ? wsum[w] : 0;
        total += wsum[w];
    }
    __syncthreads();
    return base + v;
}

__global__ void __launch_bounds__(1024)
k_scan_sums(const int64_t *__restrict__ blk, int64_t n, int64_t seg, int64_t *__restrict__ part)
{
    __shared__ int64_t wsum[16];
    const int64_t lo = (int64_t)blockIdx.x * seg, hi = min(lo + seg, n);
    int64_t sum = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 1024) sum += blk[i];
    int64_t total;
    (void)block_scan1024(sum, wsum, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024)
k_scan_parts(int64_t *part, int nparts, int nshots, int64_t *offsets, int64_t capacity,
             int64_t *status, int64_t *total_out)
{
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x;
    const int64_t v = t < nparts ? part[t] : 0;
    int64_t total;
    const int64_t incl = block_scan1024(v, wsum, total);
    if (t < nparts) part[t] = incl - v;
    if (t == 0) {
        *total_out = total;
        offsets[nshots] = min(total, capacity);
        if (total > capacity) {
            atomicOr((unsigned long long *)&status[0], FGA_STATUS_CAPACITY);
            atomicMax((unsigned long long *)&status[1], (unsigned long long)total);
        }
    }
}

__global__ void __launch_bounds__(1024)
k_scan_down(int64_t *__restrict__ blk, int64_t n, int64_t seg, const int64_t *__restrict__ part,
            int nblk, int nshots, int64_t *offsets, int64_t capacity)
{
    __shared__ int64_t wsum[16];
    const int64_t lo = (int64_t)blockIdx.x * seg, hi = min(lo + seg, n);
    int64_t run = part[blockIdx.x];
    for (int64_t t0 = lo; t0 < hi; t0 += 1024) {
        const int64_t i = t0 + threadIdx.x;
        const int64_t v = i < hi ? blk[i] : 0;
        int64_t total;
        const int64_t excl = run + block_scan1024(v, wsum, total) - v;
        if (i < hi) {
            blk[i] = excl;
            if (i % nblk == 0 && i / nblk < nshots) offsets[i / nblk] = min(excl, capacity);
        }
        run += total;
    }
}

// exclusive prefix over the workgroup of a per-round wave ballot
__device__ __forceinline__ int block_rank(unsigned long long m, int *wsum, int &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < CMP_BLOCK / 64; ++w) {
        base += w < wv ? wsum[w] : 0;
        total += wsum[w];
    }
    __syncthreads();
    return base + __popcll(m & ((1ull << lane) - 1ull));
}

// one kept beam at position pos: mesh node, coefficient, initial state, id
template <typename R>
__device__ __forceinline__ void write_beam(const fga_beams &B, int64_t pos, int64_t id, double q1,
                                           double q2, double p1, double p2, double cre,
                                           double cim)
{
    const int64_t cap = B.capacity;
    double *f = B.f;
    f[0 * cap + pos] = q1;
    f[1 * cap + pos] = q2;
    f[2 * cap + pos] = p1;
    f[3 * cap + pos] = p2;
    f[4 * cap + pos] = cre;
    f[5 * cap + pos] = cim;
    const double init[FGA_NSTATE] = {q1, q2, p1, p2, 0.0,
                                     1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0,    // A = I
                                     0.0, -1.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0,  // B = -i I
                                     2.0, 0.0};                                 // a = 2
#pragma unroll
    for (int k = 0; k < FGA_NSTATE; ++k) f[(size_t)(FGA_F_STATE + k) * cap + pos] = init[k];
    B.id[pos] = id;
}

// Compaction in candidate order: per round, wave ballots rank the tied and
// the kept candidates inside each wavefront and the wavefront totals (LDS)
// order the wavefronts, so kept beams of one round land at consecutive
// positions and ties are taken in candidate order.  With sym (f1 = 0) only
// the blocks of branch + run, and every kept candidate is also written as
// the beam of branch - at the same rank inside the matching block (same
// coefficient, same initial state, id + Nq Np).
template <typename R>
__global__ void __launch_bounds__(CMP_BLOCK)
k_scatter(const cplx<R> *__restrict__ Psi, const double *__restrict__ cq, CandGeom G,
          const Sel *sel, const int64_t *blk_pos, const int64_t *blk_tie, int nblkb,
          size_t nblk_all, const int64_t *total, fga_beams B, double o1, double o2, double d1,
          double d2, int qb1, int qb2, int qs1, int qs2, double norm, int sym)
{
    __shared__ int wsum[CMP_BLOCK / 64];
    const CmpBlock C = cmp_block(G, nblkb);
    const int s = C.s;
    const Sel S = sel[s * 2 + C.sb];
    const int64_t cap = B.capacity;
    const size_t at = (size_t)s * 2 * nblkb + blockIdx.x;
    int64_t run = blk_pos[at];
    // the block keeps what the scan gave it: most blocks keep nothing and
    // need not read their candidates again
    if ((at + 1 < nblk_all ? blk_pos[at + 1] : *total) == run) return;
    int64_t run_m = sym ? blk_pos[at + nblkb] : 0;
    int64_t tie_run = blk_tie[at];
    for (int i = 0; i < CMP_ITEMS; ++i) {
        const int64_t cl = C.first + (int64_t)i * CMP_BLOCK + threadIdx.x;
        R re = 0, im = 0;
        unsigned long long key = 0ull;
        if (cl < C.end) {
            cand_psi(Psi, cq, G, s, cl, re, im);
            key = mag_key(cabs_r(re, im));
        }
        const bool tie = key == S.key && key != 0ull;
        bool keep = key > S.key;
        if (S.ties > 0) {   // uniform over the workgroup
            int ntie = 0;
            const int tr = block_rank(__ballot(tie), wsum, ntie);
            keep = keep || (tie && tie_run + tr < S.ties);
            tie_run += ntie;
        }
        int nkeep = 0;
        const int rank = block_rank(__ballot(keep), wsum, nkeep);
        const int64_t pos = run + rank, pos_m = run_m + rank;
        run += nkeep;
        run_m += nkeep;
        if (keep && (pos < cap || (sym && pos_m < cap))) {
            int sb, j1, j2, l1, l2;
            int64_t qf;
            cand_index(G, cl, sb, qf, j1, j2, l1, l2);
            const double q1 = o1 + (qb1 + j1 * qs1) * d1, q2 = o2 + (qb2 + j2 * qs2) * d2;
            const double p1 = (l1 - 0.5 * (G.np1 - 1)) * G.dp1;
            const double p2 = (l2 - 0.5 * (G.np2 - 1)) * G.dp2;
            const double cre = norm * (double)re, cim = norm * (double)im;
            const int64_t id = (int64_t)s * G.per_shot + cl;
            if (pos < cap) write_beam<R>(B, pos, id, q1, q2, p1, p2, cre, cim);
            if (sym && pos_m < cap)
                write_beam<R>(B, pos_m, id + G.Nq * G.Np, q1, q2, p1, p2, cre, cim);
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
    if (p.top_n > 0 && 2 * nshots > 65535)
        return fga_fail(ctx, FGA_EINVAL, "top_n selection takes at most 32767 shots per call");
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
    G.small = G.Nq * G.Np < (int64_t)1 << 32;
    G.fNp = fast_div((uint32_t)std::min<int64_t>(G.Np, 0xffffffffLL));
    G.fnq1 = fast_div((uint32_t)p.nq1);
    G.fnp1 = fast_div((uint32_t)p.np1);
    G.dp1 = p.dp1;
    G.dp2 = p.dp2;
    G.eps = p.eps;
    const int64_t nblkb64 = (G.Nq * G.Np + CMP_TILE - 1) / CMP_TILE;
    if (2 * nblkb64 > 0x7fffffff) return fga_fail(ctx, FGA_EINVAL, "too many candidates per shot");
    const int nblkb = (int)nblkb64, nblk = 2 * nblkb;
    // compaction counts: kept (then positions) and equal-key counts (then tie
    // ranks) per block; the selection records and radix histograms
    const size_t nblk_all = (size_t)nshots * nblk;
    const int nsb = 2 * nshots;
    const size_t sel_bytes = (size_t)nsb * sizeof(Sel), hist_bytes = (size_t)nsb * TOPN_BINS * 8;
    const size_t sel_elems = (sel_bytes + hist_bytes + 7) / 8;
    size_t have_blk = ctx->blk_elems * sizeof(int64_t);
    if ((rc = fga_ensure(ctx, (void **)&ctx->blk, &have_blk,
                         (2 * nblk_all + sel_elems + SCAN_SEGS + 1) * sizeof(int64_t),
                         "compaction counts")) != FGA_OK)
        return rc;
    ctx->blk_elems = have_blk / sizeof(int64_t);
    int64_t *blk_kept = ctx->blk, *blk_eq = ctx->blk + nblk_all;
    Sel *sel = (Sel *)(ctx->blk + 2 * nblk_all);
    unsigned long long *hist = (unsigned long long *)((char *)sel + sel_bytes);
    int64_t *scan_part = ctx->blk + 2 * nblk_all + sel_elems;

    if (fresh) {
        hipLaunchKernelGGL(k_tables<R>, dim3(512), dim3(256), 0, st, (cplx<R> *)ctx->E1t,
                           (cplx<R> *)ctx->E2, ctx->R1, ctx->R2, p.np1, p.np2, p.dp1, p.dp2,
                           g.d1, g.d2, p.eps);
        FGA_HIP(ctx, hipGetLastError());
    }
    int nq = p.nq1 * p.nq2;
    hipLaunchKernelGGL(k_cq, dim3((nq + 255) / 256), dim3(256), 0, st, fga_velgrid(ctx), g.o1,
                       g.o2, g.d1, g.d2, p.qb1, p.qb2, p.qs1, p.qs2, p.nq1, p.nq2, ctx->cq);
    // f1 = 0: psi_+ = psi_- = psi0 / 2, so the branch maximum is folded into
    // pass 2 (relative threshold) and the compaction reads each candidate once
    // for both branches
    const int sym = nfj == 1;
    unsigned long long *fold = (sym && p.top_n == 0) ? ctx->maxbits : nullptr;
    if (fold)
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, st, ctx->maxbits, nshots);
    dim3 g1((p.np1 + P1_BN - 1) / P1_BN, (g.n2 + P1_BM - 1) / P1_BM, S * p.nq1);
    const bool split = std::is_same<R, float>::value && ctx->prec == FGA_MIXED_SPLIT;
    if (split)
        hipLaunchKernelGGL(k_zero_u32_fbi, dim3((S + 255) / 256), dim3(256), 0, st, ctx->tmax, S);
    hipLaunchKernelGGL(k_fbi_pass1<R>, g1, dim3(256), 0, st, f0, f1, nfj,
                       (const cplx<R> *)ctx->E1t, (cplx<R> *)ctx->T, g.n1, g.n2, ctx->R1, p.qb1,
                       p.qs1, p.nq1, p.np1, g.d1, split ? ctx->tmax : nullptr);
    if (split) {
        dim3 g2(p2_grid_x((int)((NC + P2M_T - 1) / P2M_T), (p.np2 + P2M_T - 1) / P2M_T), 1,
                S * p.nq2);
        hipLaunchKernelGGL(k_fbi_pass2_split, g2, dim3(256), 0, st, (const cplx<float> *)ctx->T,
                           (const cplx<float> *)ctx->E2, (cplx<float> *)ctx->Psi, g.n2, ctx->R2,
                           p.qb2, p.qs2, p.nq2, p.np2, (int)NC, g.d2, ctx->tmax, fold);
    } else if (std::is_same<R, float>::value) {
        dim3 g2(p2_grid_x((int)((NC + P2M_T - 1) / P2M_T), (p.np2 + P2M_T - 1) / P2M_T), 1,
                S * p.nq2);
        hipLaunchKernelGGL(k_fbi_pass2_mfma, g2, dim3(256), 0, st, (const cplx<float> *)ctx->T,
                           (const cplx<float> *)ctx->E2, (cplx<float> *)ctx->Psi, g.n2, ctx->R2,
                           p.qb2, p.qs2, p.nq2, p.np2, (int)NC, g.d2, fold);
    } else {
        dim3 g2((unsigned)((NC + P2D_T - 1) / P2D_T), (p.np2 + P2D_T - 1) / P2D_T, S * p.nq2);
        hipLaunchKernelGGL(k_fbi_pass2_mfma64, g2, dim3(256), 0, st,
                           (const cplx<double> *)ctx->T, (const cplx<double> *)ctx->E2,
                           (cplx<double> *)ctx->Psi, g.n2, ctx->R2, p.qb2, p.qs2, p.nq2, p.np2,
                           (int)NC, g.d2, fold);
    }
    if (p.top_n > 0) {
        const int npass = (int)sizeof(R);   // eight bits of the key per pass
        hipLaunchKernelGGL(k_topn_init, dim3((nsb * TOPN_BINS + 255) / 256), dim3(256), 0, st,
                           sel, hist, nsb, (long long)p.top_n);
        const int gh = (int)std::min<int64_t>((G.Nq * G.Np + 255) / 256, 512);
        for (int pass = 0; pass < npass; ++pass) {
            hipLaunchKernelGGL(k_topn_hist<R>, dim3(gh, nsb), dim3(256), 0, st,
                               (const cplx<R> *)ctx->Psi, ctx->cq, G, sel, hist, pass, npass);
            hipLaunchKernelGGL(k_topn_pick, dim3((nsb + 63) / 64), dim3(64), 0, st, sel, hist,
                               nsb, pass, npass);
        }
    } else {
        if (!fold) {
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, st, ctx->maxbits, nshots);
            int gmax = (int)std::min<int64_t>((G.per_shot + 255) / 256, 1024);
            hipLaunchKernelGGL(k_branch_max<R>, dim3(gmax, nshots), dim3(256), 0, st,
                               (const cplx<R> *)ctx->Psi, ctx->cq, G, ctx->maxbits);
        }
        hipLaunchKernelGGL(k_sel_threshold<R>, dim3((nsb + 63) / 64), dim3(64), 0, st,
                           ctx->maxbits, p.tau, sel, nsb);
    }
    const int nblk_run = sym ? nblkb : nblk;
    hipLaunchKernelGGL(k_count<R>, dim3(nblk_run, nshots), dim3(CMP_BLOCK), 0, st,
                       (const cplx<R> *)ctx->Psi, ctx->cq, G, sel, blk_kept, blk_eq, nblkb, sym);
    // the tie ranks matter only to the N-largest rule (the threshold takes no
    // equal keys: Sel.ties = 0)
    if (p.top_n > 0)
        hipLaunchKernelGGL(k_scan_ties, dim3(nsb), dim3(1024), 0, st, sel, blk_kept, blk_eq,
                           nblkb);
    {
        const int64_t n = (int64_t)nblk_all;
        const int64_t seg = std::max<int64_t>((n + SCAN_SEGS - 1) / SCAN_SEGS, 1024);
        const int nseg = (int)((n + seg - 1) / seg);
        hipLaunchKernelGGL(k_scan_sums, dim3(nseg), dim3(1024), 0, st, blk_kept, n, seg,
                           scan_part);
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, st, scan_part, nseg, nshots,
                           beams->offsets, beams->capacity, ctx->status, scan_part + SCAN_SEGS);
        hipLaunchKernelGGL(k_scan_down, dim3(nseg), dim3(1024), 0, st, blk_kept, n, seg,
                           (const int64_t *)scan_part, nblk, nshots, beams->offsets,
                           beams->capacity);
    }
    hipLaunchKernelGGL(k_scatter<R>, dim3(nblk_run, nshots), dim3(CMP_BLOCK), 0, st,
                       (const cplx<R> *)ctx->Psi, ctx->cq, G, sel, blk_kept, blk_eq, nblkb,
                       nblk_all, (const int64_t *)(scan_part + SCAN_SEGS), *beams, g.o1, g.o2,
                       g.d1, g.d2, p.qb1, p.qb2, p.qs1, p.qs2, ctx->norm, sym);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

fga_status fga_launch_decompose(fga_ctx *ctx, int nshots, const double *f0, const double *f1,
                                fga_beams *beams)
{
    if (ctx->prec == FGA_FP64) return decompose_impl<double>(ctx, nshots, f0, f1, beams);
    return decompose_impl<float>(ctx, nshots, f0, f1, beams);
}
