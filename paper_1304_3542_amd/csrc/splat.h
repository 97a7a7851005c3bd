// Shared pieces of the reconstruction kernels: the tile size, the kernel
// arguments, the per-beam record of the mixed splat and its per-lane factor
// and MFMA fragment code.
#pragma once

#include "fga_internal.h"

#define SP_T 64          // tile edge (nodes)
#define SP_KC 16         // beams per factor batch
#define SP_CHUNK 256     // beams scanned per pass (= block size)

struct SplatArgs {
    const double *f;
    const int64_t *offsets;
    int64_t cap;
    int n1, n2;
    double o1, o2, d1, d2;
    double eps, inv_eps, half_inv_eps;
    int Rw1, Rw2;
    int nsplit, ntile1;
    double *partial;   // [nshots][nsplit][n2][n1]
    // FGA_MIXED_SPLIT: the beams' ids, candidates per shot, and the per-shot
    // largest |C a| (FP32 bit patterns) that k_splat_prep gathers
    const int64_t *id;
    int64_t per_shot;
    unsigned *wmax;
};

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
//   theta1(x1) = (S + P1 (x1 - Q1)) / (2 pi eps) = A1 + B1 x1,
//   theta2(x2) = P2 (x2 - Q2) / (2 pi eps)       = A2 + B2 x2,
// the Gaussian centre, C a in FP32 and the truncation box.  64 bytes, read
// with one scalar load per beam.
struct __align__(64) SplatRec {
    double A1, B1, A2, B2, Q1, Q2;
    float car, cai;
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
    const float e1 = __builtin_amdgcn_exp2f(-rf1 * rf1 * hl2e);
    const float sn1 = __builtin_amdgcn_sinf(th1), cs1 = __builtin_amdgcn_cosf(th1);
    const bool in1 = i1 >= r.lo1 && i1 <= r.hi1;
    const float ur = in1 ? e1 * (r.car * cs1 - r.cai * sn1) : 0.f;
    const float nui = in1 ? -e1 * (r.car * sn1 + r.cai * cs1) : 0.f;
    const double t2 = fma(r.B2, x2, r.A2);
    const float th2 = (float)(t2 - rint(t2));
    const float rf2 = (float)(x2 - r.Q2);
    const float e2 = __builtin_amdgcn_exp2f(-rf2 * rf2 * hl2e);
    const bool in2 = i2 >= r.lo2 && i2 <= r.hi2;
    const float vr = in2 ? e2 * __builtin_amdgcn_cosf(th2) : 0.f;
    const float vi = in2 ? e2 * __builtin_amdgcn_sinf(th2) : 0.f;
    auto va = __builtin_amdgcn_permlane32_swap(__float_as_uint(vr), __float_as_uint(vi), false,
                                               false);
    auto ub = __builtin_amdgcn_permlane32_swap(__float_as_uint(ur), __float_as_uint(nui), false,
                                               false);
    return {__uint_as_float(va[0]), __uint_as_float(va[1]), __uint_as_float(ub[0]),
            __uint_as_float(ub[1])};
}

// rank-one update of the 64 x 64 tile: four MFMAs.  Blocks that the beam's
// box misses get zero factors and add exact zeros; testing for them costs
// more scalar work and branches than the matrix cores spend on them.
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
// factors at two rows and two columns (the tile's two 32-row and 32-column
// blocks); four MFMAs cover the 64 x 64 tile for two beams.  U carries
// C a e^{iS/eps} times a power of two per shot that keeps it inside the FP16
// range (|U| < 2^14); the FP64 fold divides it out exactly.
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// (x, y) -> packed FP16 hi pair and lo pair
__device__ __forceinline__ void split_pair(float x, float y, unsigned &hi, unsigned &lo)
{
    const halfx2 h = __builtin_convertvector((floatx2){x, y}, halfx2);
    hi = __builtin_bit_cast(unsigned, h);
    const float hx = (float)__builtin_bit_cast(_Float16, (unsigned short)(hi & 0xffffu));
    const float hy = (float)__builtin_bit_cast(_Float16, (unsigned short)(hi >> 16));
    const halfx2 l = __builtin_convertvector((floatx2){x - hx, y - hy}, halfx2);
    lo = __builtin_bit_cast(unsigned, l);
}

struct SplitFrags {
    unsigned vh[2], vl[2];   // rows: block a = 0, 1
    unsigned uh[2], ul[2];   // columns: block c = 0, 1
};

// Factors of one beam at the lane's two rows (x2a, x2b) and two columns
// (x1a, x1b), zeroed outside the box (or for an absent beam), split into
// FP16 hi/lo pairs.  W = C a scaled by the shot's power of two.
__device__ __forceinline__ SplitFrags beam_split(const SplatRec &r, bool valid, float wr, float wi,
                                                 int i1a, const double x1s[2], int i2a,
                                                 const double x2s[2], float hl2e)
{
    SplitFrags f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int i1 = i1a + 32 * c;
        const double x1 = x1s[c];
        const double t1 = fma(r.B1, x1, r.A1);
        const float th1 = (float)(t1 - rint(t1));
        const float rf1 = (float)(x1 - r.Q1);
        const float e1 = __builtin_amdgcn_exp2f(-rf1 * rf1 * hl2e);
        const float sn1 = __builtin_amdgcn_sinf(th1), cs1 = __builtin_amdgcn_cosf(th1);
        const bool in1 = valid && i1 >= r.lo1 && i1 <= r.hi1;
        const float ur = in1 ? e1 * (wr * cs1 - wi * sn1) : 0.f;
        const float nui = in1 ? -e1 * (wr * sn1 + wi * cs1) : 0.f;
        split_pair(ur, nui, f.uh[c], f.ul[c]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int i2 = i2a + 32 * a;
        const double x2 = x2s[a];
        const double t2 = fma(r.B2, x2, r.A2);
        const float th2 = (float)(t2 - rint(t2));
        const float rf2 = (float)(x2 - r.Q2);
        const float e2 = __builtin_amdgcn_exp2f(-rf2 * rf2 * hl2e);
        const bool in2 = valid && i2 >= r.lo2 && i2 <= r.hi2;
        const float vr = in2 ? e2 * __builtin_amdgcn_cosf(th2) : 0.f;
        const float vi = in2 ? e2 * __builtin_amdgcn_sinf(th2) : 0.f;
        split_pair(vr, vi, f.vh[a], f.vl[a]);
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

