// Shared device code of the ray / dynamic-ray-tracing / amplitude system:
// complex helpers, the 23-double beam state, the right-hand side and the
// fused RK4 stage (forward propagation and the recomputation inside the
// adjoint both use it).
#pragma once

#include "fga_internal.h"

struct Cd {
    double r, i;
};

__device__ __forceinline__ Cd cmul(Cd a, Cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ Cd cadd(Cd a, Cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ Cd csub(Cd a, Cd b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ Cd cscale(Cd a, double s) { return {a.r * s, a.i * s}; }
// acc + a b and acc - a b as FMA chains (no separate product and add)
__device__ __forceinline__ Cd cfma(Cd a, Cd b, Cd acc)
{
    return {fma(a.r, b.r, fma(-a.i, b.i, acc.r)), fma(a.r, b.i, fma(a.i, b.r, acc.i))};
}
__device__ __forceinline__ Cd cfms(Cd a, Cd b, Cd acc)
{
    return {fma(-a.r, b.r, fma(a.i, b.i, acc.r)), fma(-a.r, b.i, fma(-a.i, b.r, acc.i))};
}

// State layout (23 doubles): Q1 Q2 P1 P2 S | A11 A12 A21 A22 (re,im) |
// B11 B12 B21 B22 (re,im) | a (re,im)
struct St {
    double Q1, Q2, P1, P2, S;
    Cd A[2][2], B[2][2];
    Cd a;
};

__device__ __forceinline__ void axpy(St &o, const St &y, double h, const St &k)
{
    o.Q1 = fma(h, k.Q1, y.Q1);
    o.Q2 = fma(h, k.Q2, y.Q2);
    o.P1 = fma(h, k.P1, y.P1);
    o.P2 = fma(h, k.P2, y.P2);
    o.S = fma(h, k.S, y.S);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            o.A[j][l].r = fma(h, k.A[j][l].r, y.A[j][l].r);
            o.A[j][l].i = fma(h, k.A[j][l].i, y.A[j][l].i);
            o.B[j][l].r = fma(h, k.B[j][l].r, y.B[j][l].r);
            o.B[j][l].i = fma(h, k.B[j][l].i, y.B[j][l].i);
        }
    o.a.r = fma(h, k.a.r, y.a.r);
    o.a.i = fma(h, k.a.i, y.a.i);
}

// Reciprocal and inverse square root: hardware estimate refined by Newton
// steps to full double precision.
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// 1/sqrt(x): hardware estimate refined by two Newton steps
// r <- r + r (1 - x r^2) / 2.
__device__ __forceinline__ double rsq64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
    r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
    return r;
}

// Right-hand side.  With n = |P|, u = P/n, g = grad c, K = Hess c:
//   H_P = s c u, H_Q = s n g, H_PP = s (c/n)(I - u u^T), H_QQ = s n K,
//   H_QP = s g u^T, H_PQ = s u g^T, so the dynamic ray tracing equations
//   become rank-one updates:
//   dA_j = s[(A_j.g - (c/n) B_j.u) u + (c/n) B_j]
//   dB_j = -s[n K A_j + (B_j.u) g]
//   da   = a [ (H_P.H_Q)/H + tr(Z^{-1} dZ)/2 ],  (H_P.H_Q)/H = s u.g,
//   tr(Z^{-1} dZ) = (Z22 dZ11 - Z12 dZ21 - Z21 dZ12 + Z11 dZ22) / det Z.
__device__ __forceinline__ void rhs(const VelGrid &V, double s, const St &y, St &k)
{
    double c, g1, g2, K11, K12, K22;
    vel_eval_coef(V, y.Q1, y.Q2, c, g1, g2, K11, K12, K22);
    double n2 = y.P1 * y.P1 + y.P2 * y.P2;
    double n = sqrt(n2);
    double inv_n = rcp64(n);
    double u1 = y.P1 * inv_n, u2 = y.P2 * inv_n;
    double sc = s * c;
    double HP1 = sc * u1, HP2 = sc * u2;
    k.Q1 = HP1;
    k.Q2 = HP2;
    k.P1 = -s * n * g1;
    k.P2 = -s * n * g2;
    k.S = y.P1 * HP1 + y.P2 * HP2 - sc * n;
    double con = c * inv_n;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        Cd Ag = cadd(cscale(y.A[j][0], g1), cscale(y.A[j][1], g2));
        Cd Bu = cadd(cscale(y.B[j][0], u1), cscale(y.B[j][1], u2));
        Cd m = csub(Ag, cscale(Bu, con));
        k.A[j][0] = cscale(cadd(cscale(m, u1), cscale(y.B[j][0], con)), s);
        k.A[j][1] = cscale(cadd(cscale(m, u2), cscale(y.B[j][1], con)), s);
        // (A_j K)_k = sum_l A[j][l] K[l][k]
        Cd AK0 = cadd(cscale(y.A[j][0], K11), cscale(y.A[j][1], K12));
        Cd AK1 = cadd(cscale(y.A[j][0], K12), cscale(y.A[j][1], K22));
        k.B[j][0] = cscale(cadd(cscale(AK0, n), cscale(Bu, g1)), -s);
        k.B[j][1] = cscale(cadd(cscale(AK1, n), cscale(Bu, g2)), -s);
    }
    Cd Z[2][2], dZ[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            Z[j][l] = {y.A[j][l].r - y.B[j][l].i, y.A[j][l].i + y.B[j][l].r};
            dZ[j][l] = {k.A[j][l].r - k.B[j][l].i, k.A[j][l].i + k.B[j][l].r};
        }
    Cd det = csub(cmul(Z[0][0], Z[1][1]), cmul(Z[0][1], Z[1][0]));
    Cd num = csub(cadd(cmul(Z[1][1], dZ[0][0]), cmul(Z[0][0], dZ[1][1])),
                  cadd(cmul(Z[0][1], dZ[1][0]), cmul(Z[1][0], dZ[0][1])));
    double id2 = rcp64(det.r * det.r + det.i * det.i);
    Cd tr = cscale(cmul(num, Cd{det.r, -det.i}), id2);
    Cd fac = {s * (u1 * g1 + u2 * g2) + 0.5 * tr.r, 0.5 * tr.i};
    k.a = cmul(y.a, fac);
}

// state of beam b from a field-major array whose field 0 is Q1
__device__ __forceinline__ void load_state_raw(const double *base, int64_t cap, int64_t b, St &y)
{
    const double *p = base + b;
    y.Q1 = p[0 * cap];
    y.Q2 = p[1 * cap];
    y.P1 = p[2 * cap];
    y.P2 = p[3 * cap];
    y.S = p[4 * cap];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            y.A[j][l].r = p[(5 + 2 * (2 * j + l)) * cap];
            y.A[j][l].i = p[(6 + 2 * (2 * j + l)) * cap];
            y.B[j][l].r = p[(13 + 2 * (2 * j + l)) * cap];
            y.B[j][l].i = p[(14 + 2 * (2 * j + l)) * cap];
        }
    y.a.r = p[21 * cap];
    y.a.i = p[22 * cap];
}

// state of beam b from the beam fields
__device__ __forceinline__ void load_state(const double *f, int64_t cap, int64_t b, St &y)
{
    load_state_raw(f + (size_t)FGA_F_STATE * cap, cap, b, y);
}

__device__ __forceinline__ void store_state(double *p, int64_t cap, const St &y)
{
    p[0 * cap] = y.Q1;
    p[1 * cap] = y.Q2;
    p[2 * cap] = y.P1;
    p[3 * cap] = y.P2;
    p[4 * cap] = y.S;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            p[(5 + 2 * (2 * j + l)) * cap] = y.A[j][l].r;
            p[(6 + 2 * (2 * j + l)) * cap] = y.A[j][l].i;
            p[(13 + 2 * (2 * j + l)) * cap] = y.B[j][l].r;
            p[(14 + 2 * (2 * j + l)) * cap] = y.B[j][l].i;
        }
    p[21 * cap] = y.a.r;
    p[22 * cap] = y.a.i;
}

// Velocity source of a stage that reads the knot cell's coefficient line
// when the stage evaluates c.
struct VelDirect {
    VelGrid V;
    __device__ __forceinline__ void eval(double x1, double x2, double &c, double &c1, double &c2,
                                         double &c11, double &c12, double &c22) const
    {
        vel_eval_coef(V, x1, x2, c, c1, c2, c11, c12, c22);
    }
    __device__ __forceinline__ void prefetch(double, double) const {}
};

// One RK4 stage fused with its use: k = f(t), acc += wacc k, and unless this
// is the last stage t = y + hnext k.  Each slope component is consumed as
// soon as it is produced, so only y, acc and t stay live across the stage.
// The amplitude needs Z = A + iB of the stage input and dZ = k_A + i k_B:
// det Z is formed first, row 0 of Z is kept aside before row 0 of t is
// overwritten, and the adjugate trace is accumulated row by row.
// The position of the next evaluation of c (the next stage's, after the last
// stage the next step's first) is known once the slope of Q is; it goes to
// vel.prefetch before the rest of the stage is computed.  (The request after
// the final step is not used; a branch around it would cost more registers.)
// With AMP false the amplitude is left alone (the caller sets it from the
// closed form); its terms then drop out of the compiled stage.
template <bool LAST, class Vel, bool AMP = true>
__device__ __forceinline__ void rk_stage(Vel &vel, double s, St &t, St &acc, const St &y,
                                         double wacc, double hnext)
{
    double c, g1, g2, K11, K12, K22;
    vel.eval(t.Q1, t.Q2, c, g1, g2, K11, K12, K22);
    const double n2 = fma(t.P1, t.P1, t.P2 * t.P2);
    const double inv_n = rsq64(n2);
    const double n = n2 * inv_n;
    double u1 = t.P1 * inv_n, u2 = t.P2 * inv_n;
    double sc = s * c;
    double con = c * inv_n;
    double ug = s * (u1 * g1 + u2 * g2);   // (H_P . H_Q) / H
    {
        double kQ1 = sc * u1, kQ2 = sc * u2;
        double kP1 = -s * n * g1, kP2 = -s * n * g2;
        double kS = t.P1 * kQ1 + t.P2 * kQ2 - sc * n;
        acc.Q1 = fma(wacc, kQ1, acc.Q1);
        acc.Q2 = fma(wacc, kQ2, acc.Q2);
        acc.P1 = fma(wacc, kP1, acc.P1);
        acc.P2 = fma(wacc, kP2, acc.P2);
        acc.S = fma(wacc, kS, acc.S);
        if (LAST) vel.prefetch(acc.Q1, acc.Q2);
        if (!LAST) {
            t.Q1 = fma(hnext, kQ1, y.Q1);
            t.Q2 = fma(hnext, kQ2, y.Q2);
            vel.prefetch(t.Q1, t.Q2);
            t.P1 = fma(hnext, kP1, y.P1);
            t.P2 = fma(hnext, kP2, y.P2);
            t.S = fma(hnext, kS, y.S);
        }
    }
    Cd Z0[2] = {{t.A[0][0].r - t.B[0][0].i, t.A[0][0].i + t.B[0][0].r},
                {t.A[0][1].r - t.B[0][1].i, t.A[0][1].i + t.B[0][1].r}};
    Cd Z1[2] = {{t.A[1][0].r - t.B[1][0].i, t.A[1][0].i + t.B[1][0].r},
                {t.A[1][1].r - t.B[1][1].i, t.A[1][1].i + t.B[1][1].r}};
    const Cd det = cfms(Z0[1], Z1[0], cmul(Z0[0], Z1[1]));
    Cd num;
    // sign-folded coefficients of the rank-one updates
    double su1 = s * u1, su2 = s * u2, scon = s * con;
    double nK11 = -s * n * K11, nK12 = -s * n * K12, nK22 = -s * n * K22;
    double mg1 = -s * g1, mg2 = -s * g2;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        Cd Ag = {fma(t.A[j][0].r, g1, t.A[j][1].r * g2), fma(t.A[j][0].i, g1, t.A[j][1].i * g2)};
        Cd Bu = {fma(t.B[j][0].r, u1, t.B[j][1].r * u2), fma(t.B[j][0].i, u1, t.B[j][1].i * u2)};
        Cd m = {fma(-con, Bu.r, Ag.r), fma(-con, Bu.i, Ag.i)};
        Cd kA0 = {fma(m.r, su1, scon * t.B[j][0].r), fma(m.i, su1, scon * t.B[j][0].i)};
        Cd kA1 = {fma(m.r, su2, scon * t.B[j][1].r), fma(m.i, su2, scon * t.B[j][1].i)};
        Cd kB0 = {fma(t.A[j][0].r, nK11, fma(t.A[j][1].r, nK12, Bu.r * mg1)),
                  fma(t.A[j][0].i, nK11, fma(t.A[j][1].i, nK12, Bu.i * mg1))};
        Cd kB1 = {fma(t.A[j][0].r, nK12, fma(t.A[j][1].r, nK22, Bu.r * mg2)),
                  fma(t.A[j][0].i, nK12, fma(t.A[j][1].i, nK22, Bu.i * mg2))};
        Cd dZ0 = {kA0.r - kB0.i, kA0.i + kB0.r};
        Cd dZ1 = {kA1.r - kB1.i, kA1.i + kB1.r};
        // adjugate trace: row 0 pairs with (Z22, -Z21), row 1 with (-Z12, Z11)
        if (j == 0)
            num = cfms(Z1[0], dZ1, cmul(Z1[1], dZ0));
        else
            num = cfms(Z0[1], dZ0, cfma(Z0[0], dZ1, num));
        acc.A[j][0] = {fma(wacc, kA0.r, acc.A[j][0].r), fma(wacc, kA0.i, acc.A[j][0].i)};
        acc.A[j][1] = {fma(wacc, kA1.r, acc.A[j][1].r), fma(wacc, kA1.i, acc.A[j][1].i)};
        acc.B[j][0] = {fma(wacc, kB0.r, acc.B[j][0].r), fma(wacc, kB0.i, acc.B[j][0].i)};
        acc.B[j][1] = {fma(wacc, kB1.r, acc.B[j][1].r), fma(wacc, kB1.i, acc.B[j][1].i)};
        if (!LAST) {
            t.A[j][0] = {fma(hnext, kA0.r, y.A[j][0].r), fma(hnext, kA0.i, y.A[j][0].i)};
            t.A[j][1] = {fma(hnext, kA1.r, y.A[j][1].r), fma(hnext, kA1.i, y.A[j][1].i)};
            t.B[j][0] = {fma(hnext, kB0.r, y.B[j][0].r), fma(hnext, kB0.i, y.B[j][0].i)};
            t.B[j][1] = {fma(hnext, kB1.r, y.B[j][1].r), fma(hnext, kB1.i, y.B[j][1].i)};
        }
    }
    if (AMP) {
        // tr(Z^{-1} dZ) / 2 = num conj(det Z) / (2 |det Z|^2)
        const double hid2 = 0.5 * rcp64(fma(det.r, det.r, det.i * det.i));
        const Cd w = cmul(num, Cd{det.r, -det.i});
        Cd ka = cmul(t.a, Cd{fma(w.r, hid2, ug), w.i * hid2});
        acc.a = {fma(wacc, ka.r, acc.a.r), fma(wacc, ka.i, acc.a.i)};
        if (!LAST) t.a = {fma(hnext, ka.r, y.a.r), fma(hnext, ka.i, y.a.i)};
    }
}

// the stage with the taps read where c is evaluated
template <bool LAST>
__device__ __forceinline__ void stage(const VelGrid &V, double s, St &t, St &acc, const St &y,
                                      double wacc, double hnext)
{
    VelDirect vel{V};
    rk_stage<LAST>(vel, s, t, acc, y, wacc, hnext);
}
