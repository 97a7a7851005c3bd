// Shared pieces of the reconstruction kernels: the tile size, the kernel
// arguments, the per-beam record of the mixed splat and its per-lane factor
// and MFMA fragment code.
#pragma once

#include "fga_internal.h"

#define SP_T 64          // tile edge (nodes)
#define SP_KC 16         // beams per factor batch
#define SP_CHUNK 256     // beams scanned per pass (= block size)
#define SP64_T 128       // tile edge of the FP64 splats (nodes)
#define SP64_KC 16       // beams per FP64 factor batch

struct SplatArgs {
    const double *f;
    const int64_t *offsets;
    int64_t cap;
    int n1, n2;
    double o1, o2, d1, d2;
    double eps, inv_eps, half_inv_eps;
    int Rw1, Rw2;
    int nsplit, ntile1;
    int tile;          // tile edge of the binned splats (nodes)
    double *partial;   // [nshots][nsplit][n2][n1], or [item][tile][tile] binned
    // FGA_MIXED_SPLIT: the beams' ids, candidates per shot, and the per-shot
    // largest |C a| (FP32 bit patterns) that k_splat_prep gathers
    const int64_t *id;
    int64_t per_shot;
    unsigned *wmax;
};

// ---------------------------------------------------------------------------
// FP64 splat pieces (a workgroup of 256 threads on a 128 x 128 tile, thread
// (tx, tz) owning the nodes (X0 + tx + 16 i, Z0 + tz + 16 j), i, j < 8).
//
// The factors of beam b (none if b < 0) at the tile's coordinates,
//   U(x1) = C a e^{(i (S + P1 r1) - r1^2/2) / eps},  V(x2) = e^{(i P2 r2 - r2^2/2) / eps},
// zero outside the beam's box (CONJ_V: conj V into v), as 16 runs of 16
// nodes (8 along x1 into u, 8 along x2 into v); thread j < 16 of the beam's
// 16 forms run j: one direct
// evaluation at the run's first node in the box and then
// g(x + d) = g(x) rho(x), rho(x + d) = rho(x) e^{-d^2/eps} (exact identities
// of the Gaussian; kap1, kap2 = e^{-d^2/eps} of the two axes).
template <bool CONJ_V = false>
__device__ __forceinline__ void sp64_stage(const SplatArgs &A, int64_t b, int X0, int Z0, int j,
                                           double kap1, double kap2, double2 *u, double2 *v)
{
    const int64_t cap = A.cap;
    const int ax = j >> 3, x0 = 16 * (j & 7);
    double2 *dst = ax == 0 ? u + x0 : v + x0;
    const double kap = ax == 0 ? kap1 : kap2;
    int m0 = 1, m1 = 0;                        // empty run
    double gr = 0.0, gi = 0.0, rr = 0.0, ri = 0.0;
    if (b >= 0) {
        const double *p = A.f + b;
        const double Q1 = p[(FGA_F_STATE + 0) * cap], Q2 = p[(FGA_F_STATE + 1) * cap];
        const BeamBox bx = beam_box(Q1, Q2, A.o1, A.o2, A.d1, A.d2, A.Rw1, A.Rw2, A.n1, A.n2);
        const int start = (ax == 0 ? X0 : Z0) + x0;
        const int blo = ax == 0 ? bx.lo1 : bx.lo2, bhi = ax == 0 ? bx.hi1 : bx.hi2;
        m0 = max(blo - start, 0);
        m1 = min(bhi - start, 15);
        if (m0 <= m1) {
            const double o = ax == 0 ? A.o1 : A.o2, d = ax == 0 ? A.d1 : A.d2;
            const double Q = ax == 0 ? Q1 : Q2;
            const double P = p[(FGA_F_STATE + 2 + ax) * cap];
            const double r = (o + (start + m0) * d) - Q;
            double th = P * r, cr = 1.0, ci = 0.0;
            if (ax == 0) {
                const double ar = p[(FGA_F_STATE + 21) * cap];
                const double ai = p[(FGA_F_STATE + 22) * cap];
                const double Cr = p[4 * cap], Ci = p[5 * cap];
                cr = Cr * ar - Ci * ai;
                ci = Cr * ai + Ci * ar;
                th += p[(FGA_F_STATE + 4) * cap];
            }
            double sn, cs;
            sincos(th * A.inv_eps, &sn, &cs);
            double e = exp(-r * r * A.half_inv_eps);
            const double wr = e * cs, wi = e * sn;
            gr = cr * wr - ci * wi;
            gi = cr * wi + ci * wr;
            sincos(P * d * A.inv_eps, &sn, &cs);
            e = exp(-(r + 0.5 * d) * d * A.inv_eps);
            rr = e * cs;
            ri = e * sn;
            if (CONJ_V && ax == 1) {
                // conj V: the conjugate start and ratio give the conjugate run
                gi = -gi;
                ri = -ri;
            }
        }
    }
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) {
        if (mm < m0 || mm > m1) {
            dst[mm] = double2{0.0, 0.0};
        } else {
            dst[mm] = double2{gr, gi};
            const double t2 = gr * rr - gi * ri;
            gi = gr * ri + gi * rr;
            gr = t2;
            rr *= kap;
            ri *= kap;
        }
    }
}

// acc[i][j] += Re(U V) at the thread's 8 x 8 nodes for the kn staged beams
__device__ __forceinline__ void sp64_accumulate(const double2 (*U)[SP64_T],
                                                const double2 (*V)[SP64_T], int kn, int tx,
                                                int tz, double acc[8][8])
{
    for (int kk = 0; kk < kn; ++kk) {
        double2 u[8], v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) u[i] = U[kk][tx + 16 * i];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = V[kk][tz + 16 * j];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                acc[i][j] = fma(u[i].x, v[j].x, fma(-u[i].y, v[j].y, acc[i][j]));
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision splat on the matrix cores.
//
// One wavefront owns a 64 x 64 output tile and a run of beams that meet it.
// Per beam, lane l evaluates V at x2 = Z0 + l and U at x1 = X0 + l (phase in
// FP64 revolutions reduced to [-1/2, 1/2], then the hardware FP32 sin, cos
// and exp2), so every factor is computed once and never leaves registers.
// Re(U V) = Vr Ur + Vi (-Ui) is a K = 2 product per beam:
//   A (32 x 2, rows = x2):  A[i][0] = Vr(i), A[i][1] = Vi(i)
//   B (2 x 32, cols = x1):  B[0][j] = Ur(j), B[1][j] = -Ui(j)
// With v_mfma_f32_32x32x2f32 lane l holds A[l % 32][l / 32] and
// B[l / 32][l % 32]; the halves of the wave swap their factors once
// (xor 32) to build the two 32-row and two 32-column fragments.  Four MFMAs
// per beam cover the tile; the FP32 accumulators are folded into FP64 ones
// after at most 256 beams.
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Per-beam record of the mixed splat, formed once per reconstruction:
// phases in revolutions as affine functions of the node coordinate,
//   theta1(x1) = (S + P1 (x1 - Q1)) / (2 pi eps) + arg(C a) / (2 pi) = A1 + B1 x1,
//   theta2(x2) = P2 (x2 - Q2) / (2 pi eps)                          = A2 + B2 x2,
// the Gaussian centre, |C a| in FP32 (so that U = |C a| g1 e^{2 pi i theta1})
// and the truncation box.  64 bytes, staged with four 16-byte loads per beam.
struct __align__(64) SplatRec {
    double A1, B1, A2, B2, Q1, Q2;
    float w, pad;
    short lo1, hi1, lo2, hi2;
};

struct Frags {
    float a0, a1, b0, b1;
};

// Factors of one beam at this lane's x1 and x2 and the MFMA fragments:
// v_permlane32_swap(x, y) exchanges the upper half of x with the lower half
// of y, which turns (Vr, Vi) into the fragments of the two 32-row blocks and
// (Ur, -Ui) into those of the two 32-column blocks.
__device__ __forceinline__ Frags beam_frags(const SplatRec &r, int i1, int i2, double x1,
                                            double x2, float hl2e)
{
    // evaluated in every lane and zeroed outside the box (no branch: almost
    // always some lane of the wavefront is inside)
    const double t1 = fma(r.B1, x1, r.A1);
    const float th1 = (float)(t1 - rint(t1));
    const float rf1 = (float)(x1 - r.Q1);
    const bool in1 = i1 >= r.lo1 && i1 <= r.hi1;
    const float g1 = in1 ? __builtin_amdgcn_exp2f(-rf1 * rf1 * hl2e) * r.w : 0.f;
    const float ur = g1 * __builtin_amdgcn_cosf(th1);
    const float nui = -(g1 * __builtin_amdgcn_sinf(th1));
    const double t2 = fma(r.B2, x2, r.A2);
    const float th2 = (float)(t2 - rint(t2));
    const float rf2 = (float)(x2 - r.Q2);
    const bool in2 = i2 >= r.lo2 && i2 <= r.hi2;
    const float g2 = in2 ? __builtin_amdgcn_exp2f(-rf2 * rf2 * hl2e) : 0.f;
    const float vr = g2 * __builtin_amdgcn_cosf(th2);
    const float vi = g2 * __builtin_amdgcn_sinf(th2);
    auto va = __builtin_amdgcn_permlane32_swap(__float_as_uint(vr), __float_as_uint(vi), false,
                                               false);
    auto ub = __builtin_amdgcn_permlane32_swap(__float_as_uint(ur), __float_as_uint(nui), false,
                                               false);
    return {__uint_as_float(va[0]), __uint_as_float(va[1]), __uint_as_float(ub[0]),
            __uint_as_float(ub[1])};
}

// rank-one update of the 64 x 64 tile: four MFMAs.  Blocks that the beam's
// box misses get zero factors and add exact zeros; testing for them costs more scalar
// work and branches than the matrix cores spend on them.
__device__ __forceinline__ void tile_update(const Frags &fr, floatx16 &acc00, floatx16 &acc01,
                                            floatx16 &acc10, floatx16 &acc11)
{
    acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(fr.a0, fr.b0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(fr.a0, fr.b1, acc01, 0, 0, 0);
    acc10 = __builtin_amdgcn_mfma_f32_32x32x2f32(fr.a1, fr.b0, acc10, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(fr.a1, fr.b1, acc11, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// The same rank-one tile updates on the FP16 matrix cores (FGA_MIXED_SPLIT).
//
// Every FP32 factor x is split into x_hi = fp16(x) and x_lo = fp16(x - x_hi)
// (both rounded to nearest; x - x_hi is exact in FP32), so
// x = x_hi + x_lo to about 2^-22 relative, and the products
// (V_hi + V_lo)(U_hi + U_lo) are summed exactly by FP32 accumulation of the
// four FP16 products.  With v_mfma_f32_32x32x16_f16 lane l supplies
// A[l % 32][8 (l / 32) + t] and B[8 (l / 32) + t][l % 32] in slot t (checked
// on the device), so the lower half of the wavefront carries one beam and
// the upper half the next: per beam eight k slots, as four pairs (Re, Im),
//   A (rows x2):  (Vr, Vi)_hi, (Vr, Vi)_hi, (Vr, Vi)_lo, (Vr, Vi)_lo
//   B (cols x1):  (Ur, -Ui)_hi, (Ur, -Ui)_lo, (Ur, -Ui)_hi, (Ur, -Ui)_lo
// whose products add up to Re(U V) = Vr Ur - Vi Ui.  A lane forms its beam's
// factors at two rows and two columns 32 nodes apart (the tile's two 32-row
// and 32-column blocks); four MFMAs cover the 64 x 64 tile for two beams.
// The factors are not masked to the truncation box, which only decides the
// tiles a beam visits: beyond the box the Gaussian is below the window
// tolerance (the box is where it reaches it), so the extra terms are smaller
// than what the box already drops, and the sum moves closer to the
// untruncated one.  The per-shot scaling keeps the products exact under a
// power-of-two change of the data (the scaled U is the same).
// The second row and column take the phase of the first turned by the
// beam's rotation over 32 nodes, R = e^{2 pi i 32 B d}, which the staging
// step forms once per beam and tile: one complex product in place of a
// phase evaluation, a sine and a cosine.  U carries |C a| g1 times a power
// of two per shot that keeps it inside the FP16 range (|U| < 2^14); the FP64
// fold divides it out exactly.
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// A beam as staged for the split splat: the record's phases, its centre in
// units of sqrt(2 eps / log2 e) (so that the Gaussian is exp2 of minus a
// square), the scaled |C a| and the 32-node rotations of both axes (80
// bytes).
struct __align__(16) SplitRec {
    double A1, B1, A2, B2, Q1s, Q2s;
    float w, r1c, r1s, r2c, r2s;
    float pad[3];
};

// (x, y) -> packed FP16 hi pair and lo pair.  The lo halves come from
// v_fma_mix{lo,hi}_f16, which forms x - fp16(x) from the packed FP16 operand
// and the FP32 one in FP32 and rounds it to FP16 in one instruction.
__device__ __forceinline__ void split_pair(float x, float y, unsigned &hi, unsigned &lo)
{
    const halfx2 h = __builtin_convertvector((floatx2){x, y}, halfx2);
    hi = __builtin_bit_cast(unsigned, h);
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, -%1, 1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=&v"(lo)
        : "v"(hi), "v"(x), "v"(y));
}

struct SplitFrags {
    unsigned vh[2], vl[2];   // rows: block a = 0, 1
    unsigned uh[2], ul[2];   // columns: block c = 0, 1
};

// Factors of one beam at the lane's rows x2, x2 + 32 d2 and columns x1,
// x1 + 32 d1, split into FP16 hi/lo pairs.  w is the scaled |C a| (zero for
// an absent beam); xs_a = x_a sqrt(log2 e / (2 eps)) and d32s_a = 32 d_a in
// the same units, so the Gaussian is exp2(-(xs - Qs)^2).  The phase is
// reduced to [0, 1) revolutions (v_sin_f32 and v_cos_f32 take revolutions).
__device__ __forceinline__ SplitFrags beam_split(const SplitRec &r, float w, double x1, double x2,
                                                 double xs1, double xs2, float d32s_1,
                                                 float d32s_2)
{
    SplitFrags f;
    {
        const float th = (float)__builtin_amdgcn_fract(fma(r.B1, x1, r.A1));
        const float rf = (float)(xs1 - r.Q1s);
        const float sn = __builtin_amdgcn_sinf(th), cs = __builtin_amdgcn_cosf(th);
        const float g0 = __builtin_amdgcn_exp2f(-rf * rf) * w;
        split_pair(g0 * cs, -(g0 * sn), f.uh[0], f.ul[0]);
        const float rg = rf + d32s_1;
        const float g1 = __builtin_amdgcn_exp2f(-rg * rg) * w;
        const float cs1 = fmaf(cs, r.r1c, -sn * r.r1s), sn1 = fmaf(sn, r.r1c, cs * r.r1s);
        split_pair(g1 * cs1, -(g1 * sn1), f.uh[1], f.ul[1]);
    }
    {
        const float th = (float)__builtin_amdgcn_fract(fma(r.B2, x2, r.A2));
        const float rf = (float)(xs2 - r.Q2s);
        const float sn = __builtin_amdgcn_sinf(th), cs = __builtin_amdgcn_cosf(th);
        const float g0 = __builtin_amdgcn_exp2f(-rf * rf);
        split_pair(g0 * cs, g0 * sn, f.vh[0], f.vl[0]);
        const float rg = rf + d32s_2;
        const float g1 = __builtin_amdgcn_exp2f(-rg * rg);
        const float cs1 = fmaf(cs, r.r2c, -sn * r.r2s), sn1 = fmaf(sn, r.r2c, cs * r.r2s);
        split_pair(g1 * cs1, g1 * sn1, f.vh[1], f.vl[1]);
    }
    return f;
}

__device__ __forceinline__ halfx8 frag8(unsigned d0, unsigned d1, unsigned d2, unsigned d3)
{
    typedef unsigned uintx4 __attribute__((ext_vector_type(4)));
    return __builtin_bit_cast(halfx8, (uintx4){d0, d1, d2, d3});
}

// two beams (one per half wavefront) on the 64 x 64 tile: four MFMAs
__device__ __forceinline__ void tile_update_split(const SplitFrags &f, floatx16 &acc00,
                                                  floatx16 &acc01, floatx16 &acc10,
                                                  floatx16 &acc11)
{
    const halfx8 a0 = frag8(f.vh[0], f.vh[0], f.vl[0], f.vl[0]);
    const halfx8 a1 = frag8(f.vh[1], f.vh[1], f.vl[1], f.vl[1]);
    const halfx8 b0 = frag8(f.uh[0], f.ul[0], f.uh[0], f.ul[0]);
    const halfx8 b1 = frag8(f.uh[1], f.ul[1], f.uh[1], f.ul[1]);
    acc00 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, b0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, b1, acc01, 0, 0, 0);
    acc10 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b0, acc10, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b1, acc11, 0, 0, 0);
}
