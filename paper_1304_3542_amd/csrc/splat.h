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
