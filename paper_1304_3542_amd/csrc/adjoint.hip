// Adjoint of the receiver-trace forward on gfx950: the exact gradient of the
// discrete forward (decompose -> RK4 -> traces) of
//   J = 1/2 sum (traces - data)^2
// with respect to the velocity samples and the initial wavefield, with the
// thresholded beam set and every truncation box held fixed.
//
//  * k_trace_adjoint: one thread per beam walks the record segments
//    backwards.  Each segment is recomputed from the checkpoint written by
//    the forward (its step states go to a per-beam scratch), the trace
//    cotangent at the record is added to the state cotangent lambda, and
//    lambda is pulled back through every RK4 step with the hand-written
//    vector-Jacobian product of the right-hand side.  dJ/dc reaches the
//    velocity samples through the B-spline tap weights (FP64 atomics);
//    dJ/dC per beam is returned for the decomposition adjoint.
//  * fga_decompose_adjoint: dJ/dpsi_{+-} = w/(2 pi eps)^3 dJ/dC, pulled back
//    through u_{+-,0} to dJ/dpsi_0 (and dJ/dpsi_1, dJ/dc(q) when f1 was
//    given), then through the two windowed DFT passes in transpose.
#include <math.h>

#include <algorithm>

#include "rk4.h"

__device__ __forceinline__ Cd cconj(Cd a) { return {a.r, -a.i}; }
// a * conj(b)
__device__ __forceinline__ Cd cmulc(Cd a, Cd b) { return {a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i}; }
// Re(conj(a) b)
__device__ __forceinline__ double cdotr(Cd a, Cd b) { return a.r * b.r + a.i * b.i; }
// -i z
__device__ __forceinline__ Cd cmuli_neg(Cd z) { return {z.i, -z.r}; }

__device__ __forceinline__ void st_zero(St &z)
{
    z.Q1 = z.Q2 = z.P1 = z.P2 = z.S = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) z.A[j][l] = z.B[j][l] = Cd{0.0, 0.0};
    z.a = Cd{0.0, 0.0};
}

// o = x + h y
__device__ __forceinline__ St st_axpy(const St &x, double h, const St &y)
{
    St o;
    axpy(o, x, h, y);
    return o;
}

// Velocity with third derivatives, and the per-axis tap factors
// (w, dw/d, ddw/d^2) for the scatter of dJ/d(c, grad c, Hess c) to samples.
struct Vel3 {
    double c, g1, g2, K11, K12, K22, T111, T112, T122, T222;
    double ax[3][4], az[3][4];
    int i1, i2;
};

__device__ __forceinline__ void vel_eval3(const VelGrid &V, double x1, double x2, Vel3 &o)
{
    double t1 = (x1 - V.o1) * V.inv_d1, t2 = (x2 - V.o2) * V.inv_d2;
    double fl1 = floor(t1), fl2 = floor(t2);
    double f1 = t1 - fl1, f2 = t2 - fl2;
    o.i1 = (int)fmin(fmax(fl1, -4.0), (double)V.n1 + 3.0);
    o.i2 = (int)fmin(fmax(fl2, -4.0), (double)V.n2 + 3.0);
    double wx[4], dwx[4], ddwx[4], wz[4], dwz[4], ddwz[4];
    bspline_w(f1, wx, dwx, ddwx);
    bspline_w(f2, wz, dwz, ddwz);
    const double dddw[4] = {-1.0, 3.0, -3.0, 1.0};
    const double *base = V.c + (size_t)(o.i2 - 1 + FGA_VPAD) * V.ld + (o.i1 - 1 + FGA_VPAD);
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
        const double *row = base + kz * V.ld;
        double v0 = row[0], v1 = row[1], v2 = row[2], v3 = row[3];
        double a0 = wx[0] * v0 + wx[1] * v1 + wx[2] * v2 + wx[3] * v3;
        double a1 = dwx[0] * v0 + dwx[1] * v1 + dwx[2] * v2 + dwx[3] * v3;
        double a2 = ddwx[0] * v0 + ddwx[1] * v1 + ddwx[2] * v2 + ddwx[3] * v3;
        double a3 = dddw[0] * v0 + dddw[1] * v1 + dddw[2] * v2 + dddw[3] * v3;
        s[0] += wz[kz] * a0;
        s[1] += wz[kz] * a1;
        s[2] += dwz[kz] * a0;
        s[3] += wz[kz] * a2;
        s[4] += dwz[kz] * a1;
        s[5] += ddwz[kz] * a0;
        s[6] += wz[kz] * a3;
        s[7] += dwz[kz] * a2;
        s[8] += ddwz[kz] * a1;
        s[9] += dddw[kz] * a0;
    }
    const double i1d = V.inv_d1, i2d = V.inv_d2;
    o.c = s[0];
    o.g1 = s[1] * i1d;
    o.g2 = s[2] * i2d;
    o.K11 = s[3] * i1d * i1d;
    o.K12 = s[4] * i1d * i2d;
    o.K22 = s[5] * i2d * i2d;
    o.T111 = s[6] * i1d * i1d * i1d;
    o.T112 = s[7] * i1d * i1d * i2d;
    o.T122 = s[8] * i1d * i2d * i2d;
    o.T222 = s[9] * i2d * i2d * i2d;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        o.ax[0][k] = wx[k];
        o.ax[1][k] = dwx[k] * i1d;
        o.ax[2][k] = ddwx[k] * i1d * i1d;
        o.az[0][k] = wz[k];
        o.az[1][k] = dwz[k] * i2d;
        o.az[2][k] = ddwz[k] * i2d * i2d;
    }
}

// Per-thread accumulator of dJ/d(samples) over the 4 x 4 knots of one cell:
// contributions are summed in place while the ray stays in the cell and the
// sums go to the grid with atomics only when the cell changes.
struct DcAcc {
    double v[16];
    int i1, i2;   // knot base of the held sums (i1 = INT_MIN: empty)
    int64_t b;    // the beam (slot of its log in deterministic mode)
    int cnt;      // records logged so far
};

// Where dJ/dc goes: added to dc with FP64 atomics (rec = null), or logged in
// the beam's own slots as records of one knot cell's 16 sums,
// rec[k][cap][16] (a record is one 128-byte line) and
// cell[k][cap] = (i2 + 4)(n1 + 8) + (i1 + 4) for the k-th logged flush of
// beam b.  Past R records a deterministic log (dc = null)
// only counts (the caller reruns with the length found); a non-deterministic
// one (dc set) adds the rest with atomics, and its count stops at R.
struct DcOut {
    double *dc;
    double *rec;
    int *cell;
    int64_t cap;
    int R, n1, n2;
};

__device__ __forceinline__ void dcacc_init(DcAcc &a, int64_t b = 0)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) a.v[k] = 0.0;
    a.i1 = -2147483647 - 1;
    a.i2 = 0;
    a.b = b;
    a.cnt = 0;
}

__device__ __forceinline__ void dcacc_flush(DcAcc &a, const DcOut &o)
{
    if (a.i1 == -2147483647 - 1) return;
    if (o.rec && (a.cnt < o.R || !o.dc)) {
        if (a.cnt < o.R) {
            double2 *r = (double2 *)(o.rec + ((size_t)a.cnt * o.cap + a.b) * 16);
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = make_double2(a.v[2 * k], a.v[2 * k + 1]);
            o.cell[(size_t)a.cnt * o.cap + a.b] = (a.i2 + 4) * (o.n1 + 8) + (a.i1 + 4);
        }
        ++a.cnt;
#pragma unroll
        for (int k = 0; k < 16; ++k) a.v[k] = 0.0;
    } else {
#pragma unroll
        for (int kz = 0; kz < 4; ++kz) {
            int r = min(max(a.i2 - 1 + kz, 0), o.n2 - 1);
#pragma unroll
            for (int kx = 0; kx < 4; ++kx) {
                int q = min(max(a.i1 - 1 + kx, 0), o.n1 - 1);
                if (a.v[4 * kz + kx] != 0.0)
                    atomicAdd(&o.dc[(size_t)r * o.n1 + q], a.v[4 * kz + kx]);
                a.v[4 * kz + kx] = 0.0;
            }
        }
    }
    a.i1 = -2147483647 - 1;
}

// acc += d(c, g1, g2, K11, K12, K22)/d(samples)^T vb at the knots of v
__device__ __forceinline__ void scatter_dc(const Vel3 &v, const double vb[6], DcAcc &acc,
                                           const DcOut &out)
{
    if (v.i1 != acc.i1 || v.i2 != acc.i2) {
        dcacc_flush(acc, out);
        acc.i1 = v.i1;
        acc.i2 = v.i2;
    }
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
        double px0 = vb[0] * v.az[0][kz] + vb[2] * v.az[1][kz] + vb[5] * v.az[2][kz];
        double px1 = vb[1] * v.az[0][kz] + vb[4] * v.az[1][kz];
        double px2 = vb[3] * v.az[0][kz];
#pragma unroll
        for (int kx = 0; kx < 4; ++kx)
            acc.v[4 * kz + kx] += px0 * v.ax[0][kx] + px1 * v.ax[1][kx] + px2 * v.ax[2][kx];
    }
}

// xb += (df/dx)^T kb, dc += (df/dc)^T kb, for k = f(x) the right-hand side
// of rk4.h.  The action slope is identically zero as a function of the
// state (H is homogeneous of degree one in P), so it carries no cotangent.
__device__ void rhs_vjp(const VelGrid &V, double s, const St &x, const St &kb, St &xb, DcAcc &dacc,
                        const DcOut &out)
{
    // ---- forward quantities
    Vel3 v;
    vel_eval3(V, x.Q1, x.Q2, v);
    const double c = v.c, g[2] = {v.g1, v.g2};
    const double K[2][2] = {{v.K11, v.K12}, {v.K12, v.K22}};
    const double n = sqrt(x.P1 * x.P1 + x.P2 * x.P2);
    const double inv_n = rcp64(n);
    const double u[2] = {x.P1 * inv_n, x.P2 * inv_n};
    const double con = c * inv_n;
    Cd Ag[2], Bu[2], m[2], AK[2][2], kA[2][2], kB[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        Ag[j] = cadd(cscale(x.A[j][0], g[0]), cscale(x.A[j][1], g[1]));
        Bu[j] = cadd(cscale(x.B[j][0], u[0]), cscale(x.B[j][1], u[1]));
        m[j] = csub(Ag[j], cscale(Bu[j], con));
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            AK[j][k] = cadd(cscale(x.A[j][0], K[0][k]), cscale(x.A[j][1], K[1][k]));
            kA[j][k] = cscale(cadd(cscale(m[j], u[k]), cscale(x.B[j][k], con)), s);
            kB[j][k] = cscale(cadd(cscale(AK[j][k], n), cscale(Bu[j], g[k])), -s);
        }
    }
    Cd Z[2][2], dZ[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            Z[j][k] = {x.A[j][k].r - x.B[j][k].i, x.A[j][k].i + x.B[j][k].r};
            dZ[j][k] = {kA[j][k].r - kB[j][k].i, kA[j][k].i + kB[j][k].r};
        }
    const Cd det = csub(cmul(Z[0][0], Z[1][1]), cmul(Z[0][1], Z[1][0]));
    const Cd num = csub(cadd(cmul(Z[1][1], dZ[0][0]), cmul(Z[0][0], dZ[1][1])),
                        cadd(cmul(Z[0][1], dZ[1][0]), cmul(Z[1][0], dZ[0][1])));
    const double id2 = rcp64(det.r * det.r + det.i * det.i);
    const Cd inv_det = cscale(cconj(det), id2);
    const Cd tr = cmul(num, inv_det);
    const double ug = u[0] * g[0] + u[1] * g[1];
    const Cd h = {s * ug + 0.5 * tr.r, 0.5 * tr.i};

    // ---- reverse
    // ka = a h
    xb.a = cadd(xb.a, cmulc(kb.a, h));
    const Cd hb = cmulc(kb.a, x.a);
    const double ugb = s * hb.r;
    const Cd trb = cscale(hb, 0.5);
    // tr = num / det
    const Cd numb = cmulc(trb, inv_det);                 // trb / conj(det)
    const Cd detb = cscale(cmulc(trb, cmul(tr, inv_det)), -1.0);   // -trb conj(tr/det)
    Cd dZb[2][2], Zb[2][2];
    dZb[0][0] = cmulc(numb, Z[1][1]);
    dZb[1][1] = cmulc(numb, Z[0][0]);
    dZb[1][0] = cscale(cmulc(numb, Z[0][1]), -1.0);
    dZb[0][1] = cscale(cmulc(numb, Z[1][0]), -1.0);
    Zb[1][1] = cadd(cmulc(numb, dZ[0][0]), cmulc(detb, Z[0][0]));
    Zb[0][0] = cadd(cmulc(numb, dZ[1][1]), cmulc(detb, Z[1][1]));
    Zb[0][1] = cscale(cadd(cmulc(numb, dZ[1][0]), cmulc(detb, Z[1][0])), -1.0);
    Zb[1][0] = cscale(cadd(cmulc(numb, dZ[0][1]), cmulc(detb, Z[0][1])), -1.0);

    double ub[2] = {ugb * g[0], ugb * g[1]};
    double gbv[2] = {ugb * u[0], ugb * u[1]};
    double nb = 0.0, conb = 0.0, cb = 0.0, K11b = 0.0, K12b = 0.0, K22b = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        Cd kAb[2], kBb[2], Ab[2], Bb[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            // Z = A + iB and dZ = kA + i kB
            Ab[k] = Zb[j][k];
            Bb[k] = cmuli_neg(Zb[j][k]);
            kAb[k] = cadd(kb.A[j][k], dZb[j][k]);
            kBb[k] = cadd(kb.B[j][k], cmuli_neg(dZb[j][k]));
        }
        // kB[j][k] = -s (n AK_j[k] + Bu_j g_k)
        Cd AKb[2];
        Cd Bub = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            AKb[k] = cscale(kBb[k], -s * n);
            nb += -s * cdotr(AK[j][k], kBb[k]);
            Bub = cadd(Bub, cscale(kBb[k], -s * g[k]));
            gbv[k] += -s * cdotr(Bu[j], kBb[k]);
        }
        // AK_j[k] = sum_l A[j][l] K[l][k]
#pragma unroll
        for (int l = 0; l < 2; ++l)
            Ab[l] = cadd(Ab[l], cadd(cscale(AKb[0], K[l][0]), cscale(AKb[1], K[l][1])));
        K11b += cdotr(x.A[j][0], AKb[0]);
        K12b += cdotr(x.A[j][0], AKb[1]) + cdotr(x.A[j][1], AKb[0]);
        K22b += cdotr(x.A[j][1], AKb[1]);
        // kA[j][k] = s (m_j u_k + con B[j][k])
        Cd mb = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            mb = cadd(mb, cscale(kAb[k], s * u[k]));
            ub[k] += s * cdotr(m[j], kAb[k]);
            conb += s * cdotr(x.B[j][k], kAb[k]);
            Bb[k] = cadd(Bb[k], cscale(kAb[k], s * con));
        }
        // m_j = Ag_j - con Bu_j
        const Cd Agb = mb;
        conb += -cdotr(Bu[j], mb);
        Bub = cadd(Bub, cscale(mb, -con));
        // Bu_j = sum_l B[j][l] u_l ; Ag_j = sum_l A[j][l] g_l
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            Bb[l] = cadd(Bb[l], cscale(Bub, u[l]));
            ub[l] += cdotr(x.B[j][l], Bub);
            Ab[l] = cadd(Ab[l], cscale(Agb, g[l]));
            gbv[l] += cdotr(x.A[j][l], Agb);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            xb.A[j][k] = cadd(xb.A[j][k], Ab[k]);
            xb.B[j][k] = cadd(xb.B[j][k], Bb[k]);
        }
    }
    // con = c / n
    cb += conb * inv_n;
    nb += -conb * c * inv_n * inv_n;
    // kP = -s n g
    nb += -s * (g[0] * kb.P1 + g[1] * kb.P2);
    gbv[0] += -s * n * kb.P1;
    gbv[1] += -s * n * kb.P2;
    // kQ = s c u
    cb += s * (u[0] * kb.Q1 + u[1] * kb.Q2);
    ub[0] += s * c * kb.Q1;
    ub[1] += s * c * kb.Q2;
    // u = P / n, n = |P|
    nb += -(ub[0] * u[0] + ub[1] * u[1]) * inv_n;
    xb.P1 += ub[0] * inv_n + nb * u[0];
    xb.P2 += ub[1] * inv_n + nb * u[1];
    // (c, g, K) = B-spline(Q; samples)
    xb.Q1 += cb * v.g1 + gbv[0] * v.K11 + gbv[1] * v.K12 + K11b * v.T111 + K12b * v.T112 +
             K22b * v.T122;
    xb.Q2 += cb * v.g2 + gbv[0] * v.K12 + gbv[1] * v.K22 + K11b * v.T112 + K12b * v.T122 +
             K22b * v.T222;
    const double vb[6] = {cb, gbv[0], gbv[1], K11b, K12b, K22b};
    scatter_dc(v, vb, dacc, out);
}

__device__ __forceinline__ St st_scale(double h, const St &x)
{
    St z;
    st_zero(z);
    return st_axpy(z, h, x);
}

// Per-thread stash of the three recomputed stage inputs y2, y3, y4 in LDS:
// [3][NSTATE][ADJ_BLOCK] per workgroup, thread index fastest.
#define ADJ_BLOCK 128

__device__ __forceinline__ void stash_put(double *st, int i, const St &x)
{
    double *p = st + (size_t)i * FGA_NSTATE * ADJ_BLOCK;
    p[0 * ADJ_BLOCK] = x.Q1;
    p[1 * ADJ_BLOCK] = x.Q2;
    p[2 * ADJ_BLOCK] = x.P1;
    p[3 * ADJ_BLOCK] = x.P2;
    p[4 * ADJ_BLOCK] = x.S;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            p[(5 + 2 * (2 * j + l)) * ADJ_BLOCK] = x.A[j][l].r;
            p[(6 + 2 * (2 * j + l)) * ADJ_BLOCK] = x.A[j][l].i;
            p[(13 + 2 * (2 * j + l)) * ADJ_BLOCK] = x.B[j][l].r;
            p[(14 + 2 * (2 * j + l)) * ADJ_BLOCK] = x.B[j][l].i;
        }
    p[21 * ADJ_BLOCK] = x.a.r;
    p[22 * ADJ_BLOCK] = x.a.i;
}

__device__ __forceinline__ void stash_get(const double *st, int i, St &x)
{
    const double *p = st + (size_t)i * FGA_NSTATE * ADJ_BLOCK;
    x.Q1 = p[0 * ADJ_BLOCK];
    x.Q2 = p[1 * ADJ_BLOCK];
    x.P1 = p[2 * ADJ_BLOCK];
    x.P2 = p[3 * ADJ_BLOCK];
    x.S = p[4 * ADJ_BLOCK];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            x.A[j][l].r = p[(5 + 2 * (2 * j + l)) * ADJ_BLOCK];
            x.A[j][l].i = p[(6 + 2 * (2 * j + l)) * ADJ_BLOCK];
            x.B[j][l].r = p[(13 + 2 * (2 * j + l)) * ADJ_BLOCK];
            x.B[j][l].i = p[(14 + 2 * (2 * j + l)) * ADJ_BLOCK];
        }
    x.a.r = p[21 * ADJ_BLOCK];
    x.a.i = p[22 * ADJ_BLOCK];
}

// lambda <- (d y_{n+1} / d y_n)^T lambda for one classical RK4 step from y:
// the stage inputs y2, y3, y4 are recomputed into the stash, then the four
// stages are pulled back in reverse order,
//   kbar_i = b_i dt lambda + a_{i+1,i} dt xbar_{i+1},  lambda' = lambda + sum xbar_i.
// The stages run as loops that are not unrolled, so one copy of the
// right-hand side and of its VJP is compiled and their live ranges do not
// pile up.
__device__ void step_vjp(const VelGrid &V, double s, const St &y, St &lam, double dt,
                         double *stash, DcAcc &dacc, const DcOut &out)
{
    const double ca[3] = {0.5 * dt, 0.5 * dt, dt};   // y_{i+2} = y + ca[i] k_{i+1}
    St x = y;
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
        St k;
        rhs(V, s, x, k);
        x = st_axpy(y, ca[i], k);
        stash_put(stash, i, x);
    }
    const double wl[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};   // weight of lambda
    const double wx[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};             // weight of xbar_{i+2}
    St yb = lam, xb;
    st_zero(xb);
#pragma unroll 1
    for (int i = 3; i >= 0; --i) {
        const St kbar = st_axpy(st_scale(wl[i], lam), wx[i], xb);
        if (i > 0)
            stash_get(stash, i - 1, x);
        else
            x = y;
        st_zero(xb);
        rhs_vjp(V, s, x, kbar, xb, dacc, out);
        yb = st_axpy(yb, 1.0, xb);
    }
    lam = yb;
}

struct TraceAdjArgs {
    VelGrid V;
    const double *f;          // beams (coefficients)
    const int64_t *id;
    const int64_t *offsets;
    int nshots;
    int64_t cap, NqNp;
    const int32_t *rec;
    int nrec, rec_every, nrec_t;
    const double *ckpt;       // [nrec_t][NSTATE][cap]
    const double *gtr;        // [nshots][nrec_t][nrec]
    double *scratch;          // [rec_every][NSTATE][cap]
    DcOut out;                // dJ/dc: atomics into [n2][n1], or the per-beam logs
    int *logcnt;              // with logs: [cap] log length per beam
    double *gcoef;            // [2][cap] (may be null)
    const int *rshape;        // receivers: {1, first column, row} for one run of a row, else 0
    const double *lam0;       // [NSTATE][cap]: cotangent of the final state (may be null)
    double *lam_out;          // [NSTATE][cap]: cotangent of the initial state (may be null)
    int n1, n2;
    double o1, o2, d1, d2, eps, dt;
    int Rw1, Rw2;
};

// e^{(g + i th) / eps}
__device__ __forceinline__ Cd gauss_phase(double th, double g, double inv_eps)
{
    double sn, cs;
    sincos(th * inv_eps, &sn, &cs);
    const double e = exp(g * inv_eps);
    return {e * cs, e * sn};
}

// EVERY: the checkpoints hold the state before every step (and the final
// one), ckpt[nrec_t * rec_every + 1][NSTATE][cap]; the segments are read,
// not recomputed, and no scratch is used.
template <bool EVERY>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_trace_adjoint(TraceAdjArgs A)
{
    __shared__ double stash_all[3 * FGA_NSTATE * ADJ_BLOCK];
    double *stash = stash_all + threadIdx.x;
    const int64_t nb = A.offsets[A.nshots];
    const int64_t cap = A.cap;
    const double inv_eps = 1.0 / A.eps;
    const int run = A.nrec > 0 ? A.rshape[0] : 0;
    const int run1 = A.nrec > 0 ? A.rshape[1] : 0, run2 = A.nrec > 0 ? A.rshape[2] : 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t idb = A.id[b];
        const double s = ((idb / A.NqNp) & 1) ? -1.0 : 1.0;
        const int shot = (int)(idb / (2 * A.NqNp));
        const Cd C = {A.f[4 * cap + b], A.f[5 * cap + b]};
        St lam;
        st_zero(lam);
        if (A.lam0) load_state_raw(A.lam0, cap, b, lam);
        Cd gC = {0.0, 0.0};
        DcAcc dacc;
        dcacc_init(dacc, b);
        for (int k = A.nrec_t - 1; k >= 0; --k) {
            St y;
            if (EVERY) {
                // the state at the record, stored by the forward
                load_state_raw(A.ckpt + (size_t)(k + 1) * A.rec_every * FGA_NSTATE * cap, cap, b,
                               y);
            } else {
                // recompute the segment from its checkpoint
                load_state_raw(A.ckpt + (size_t)k * FGA_NSTATE * cap, cap, b, y);
                for (int j = 0; j < A.rec_every; ++j) {
                    store_state(A.scratch + (size_t)j * FGA_NSTATE * cap + b, cap, y);
                    St t = y, acc = y;
                    stage<false>(A.V, s, t, acc, y, A.dt / 6.0, 0.5 * A.dt);
                    stage<false>(A.V, s, t, acc, y, A.dt / 3.0, 0.5 * A.dt);
                    stage<false>(A.V, s, t, acc, y, A.dt / 3.0, A.dt);
                    stage<true>(A.V, s, t, acc, y, A.dt / 6.0, 0.0);
                    y = acc;
                }
            }
            // cotangent of the traces of record k (boxes held fixed).  The
            // traced term of receiver x is Re(C a e(x)), e = e^{(i (S + P.r)
            // - |r|^2 / 2) / eps}, r = x - Q, so with F = sum R e,
            // F_k = sum R r_k e over the receivers in the box every
            // derivative follows from F, F_1, F_2.
            if (A.nrec > 0) {
                const double *R = A.gtr + ((size_t)shot * A.nrec_t + k) * A.nrec;
                const BeamBox bx =
                    beam_box(y.Q1, y.Q2, A.o1, A.o2, A.d1, A.d2, A.Rw1, A.Rw2, A.n1, A.n2);
                Cd F0 = {0.0, 0.0}, F1 = {0.0, 0.0}, F2 = {0.0, 0.0};
                if (run) {
                    // one row: e at the next column is e times rho, and rho
                    // itself steps by the real factor e^{-d1^2 / eps}
                    const int a1 = max(bx.lo1, run1), b1 = min(bx.hi1, run1 + A.nrec - 1);
                    if (run2 >= bx.lo2 && run2 <= bx.hi2 && a1 <= b1) {
                        const double r2 = (A.o2 + run2 * A.d2) - y.Q2;
                        const double r1a = (A.o1 + a1 * A.d1) - y.Q1;
                        Cd e = gauss_phase(y.S + y.P1 * r1a + y.P2 * r2,
                                           -0.5 * (r1a * r1a + r2 * r2), inv_eps);
                        Cd rho = gauss_phase(y.P1 * A.d1, -(r1a + 0.5 * A.d1) * A.d1, inv_eps);
                        const double kap = exp(-A.d1 * A.d1 * inv_eps);
                        for (int i1 = a1; i1 <= b1; ++i1) {
                            const double Rv = R[i1 - run1];
                            const double r1 = (A.o1 + i1 * A.d1) - y.Q1;
                            F0 = cadd(F0, cscale(e, Rv));
                            F1 = cadd(F1, cscale(e, Rv * r1));
                            e = cmul(e, rho);
                            rho = cscale(rho, kap);
                        }
                        F2 = cscale(F0, r2);
                    }
                } else {
                    for (int r = 0; r < A.nrec; ++r) {
                        const int node = A.rec[r];
                        const int i1 = node % A.n1, i2 = node / A.n1;
                        if (i1 < bx.lo1 || i1 > bx.hi1 || i2 < bx.lo2 || i2 > bx.hi2) continue;
                        const double r1 = (A.o1 + i1 * A.d1) - y.Q1;
                        const double r2 = (A.o2 + i2 * A.d2) - y.Q2;
                        const Cd e = gauss_phase(y.S + y.P1 * r1 + y.P2 * r2,
                                                 -0.5 * (r1 * r1 + r2 * r2), inv_eps);
                        const double Rv = R[r];
                        F0 = cadd(F0, cscale(e, Rv));
                        F1 = cadd(F1, cscale(e, Rv * r1));
                        F2 = cadd(F2, cscale(e, Rv * r2));
                    }
                }
                const Cd Ca = cmul(C, y.a);
                const Cd E0 = cmul(Ca, F0), E1 = cmul(Ca, F1), E2 = cmul(Ca, F2);
                gC = cadd(gC, cconj(cmul(y.a, F0)));
                lam.a = cadd(lam.a, cconj(cmul(C, F0)));
                lam.S += -E0.i * inv_eps;
                lam.P1 += -E1.i * inv_eps;
                lam.P2 += -E2.i * inv_eps;
                lam.Q1 += (E0.i * y.P1 + E1.r) * inv_eps;
                lam.Q2 += (E0.i * y.P2 + E2.r) * inv_eps;
            }
            // pull lambda back through the segment
            for (int j = A.rec_every - 1; j >= 0; --j) {
                St yj;
                if (EVERY)
                    load_state_raw(A.ckpt + ((size_t)k * A.rec_every + j) * FGA_NSTATE * cap, cap,
                                   b, yj);
                else
                    load_state_raw(A.scratch + (size_t)j * FGA_NSTATE * cap, cap, b, yj);
                step_vjp(A.V, s, yj, lam, A.dt, stash, dacc, A.out);
            }
        }
        dcacc_flush(dacc, A.out);
        if (A.logcnt) A.logcnt[b] = dacc.cnt;
        if (A.gcoef) {
            A.gcoef[b] = gC.r;
            A.gcoef[cap + b] = gC.i;
        }
        if (A.lam_out) store_state(A.lam_out + b, cap, lam);
    }
}

// Log slots per beam of a non-deterministic adjoint call (0: no logs).
static int grad_log_slots(const fga_ctx *ctx, int64_t cap, int64_t steps)
{
    const int64_t most = 4 * steps + 1;   // a flush per stage at most, and the last
    if (ctx->p.grad_log < 0 || cap <= 0) return 0;
    if (ctx->p.grad_log > 0) return (int)std::min<int64_t>(ctx->p.grad_log, most);
    const int64_t per = (int64_t)(16 * sizeof(double) + sizeof(int));
    // at most FGA_GRAD_LOG_BYTES, and at most half of the device memory that
    // is free (counting the logs this context holds already)
    int64_t budget = FGA_GRAD_LOG_BYTES;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
        budget = std::min<int64_t>(budget, (int64_t)(free_b / 2 + ctx->det_log_bytes));
    else
        (void)hipGetLastError();
    const int64_t fit = (budget - cap * (int64_t)sizeof(int)) / (per * cap);
    return (int)std::max<int64_t>(0, std::min<int64_t>(most, fit));
}

fga_status fga_launch_trace_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                    const int32_t *rec, int nrec, int rec_every, int nrec_t,
                                    const double *ckpt, const double *gtr, double *dc,
                                    double *gcoef)
{
    return fga_launch_rk4_adjoint(ctx, beams, nshots, rec, nrec, rec_every, nrec_t, ckpt, gtr, dc,
                                  gcoef, nullptr, nullptr);
}

// The pull-back through nseg segments of seg RK4 steps (the checkpoints hold
// the states at the segment starts), with the receiver cotangents of every
// record (nrec > 0) and/or an initial cotangent lam0 of the final state;
// lam_out receives the cotangent of the initial state.
fga_status fga_launch_rk4_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                  const int32_t *rec, int nrec, int rec_every, int nrec_t,
                                  const double *ckpt, const double *gtr, double *dc,
                                  double *gcoef, const double *lam0, double *lam_out)
{
    const int64_t cap = beams->capacity;
    const bool every = ctx->p.ckpt_every_step != 0;
    fga_status rc = FGA_OK;
    if (!every) {
        const size_t need = (size_t)rec_every * FGA_NSTATE * cap * sizeof(double);
        rc = fga_ensure(ctx, &ctx->adj_scratch, &ctx->adj_scratch_bytes, need,
                        "adjoint segment scratch");
        if (rc != FGA_OK) return rc;
    }
    auto kernel = every ? k_trace_adjoint<true> : k_trace_adjoint<false>;
    TraceAdjArgs A;
    A.V = fga_velgrid(ctx);
    A.f = beams->f;
    A.id = beams->id;
    A.offsets = beams->offsets;
    A.nshots = nshots;
    A.cap = cap;
    A.NqNp = (int64_t)ctx->p.nq1 * ctx->p.nq2 * ctx->p.np1 * ctx->p.np2;
    A.rec = rec;
    A.nrec = nrec;
    A.rec_every = rec_every;
    A.nrec_t = nrec_t;
    A.ckpt = ckpt;
    A.gtr = gtr;
    A.scratch = (double *)ctx->adj_scratch;
    A.out = DcOut{dc, nullptr, nullptr, cap, 0, ctx->g.n1, ctx->g.n2};
    A.logcnt = nullptr;
    A.gcoef = gcoef;
    A.lam0 = lam0;
    A.lam_out = lam_out;
    A.rshape = nullptr;
    if (nrec > 0) {
        rc = fga_rec_shape(ctx, rec, nrec, &A.rshape);
        if (rc != FGA_OK) return rc;
    }
    A.n1 = ctx->g.n1;
    A.n2 = ctx->g.n2;
    A.o1 = ctx->g.o1;
    A.o2 = ctx->g.o2;
    A.d1 = ctx->g.d1;
    A.d2 = ctx->g.d2;
    A.eps = ctx->p.eps;
    A.dt = ctx->p.dt;
    A.Rw1 = ctx->Rw1;
    A.Rw2 = ctx->Rw2;
    const dim3 grid(ctx->num_cu * 4), block(ADJ_BLOCK);
    const int64_t steps = (int64_t)rec_every * nrec_t;
    if (!ctx->p.deterministic) {
        int R = grad_log_slots(ctx, cap, steps);
        char *base = nullptr;
        size_t rec_bytes = 0, cell_bytes = 0;
        if (R > 0) {
            rec_bytes = (size_t)R * 16 * cap * sizeof(double);
            cell_bytes = (size_t)R * cap * sizeof(int);
            rc = fga_ensure(ctx, &ctx->det_log, &ctx->det_log_bytes,
                            rec_bytes + cell_bytes + (size_t)cap * sizeof(int), "dJ/dc logs");
            if (rc == FGA_ENOMEM) {
                // no room for the logs: every record goes to dc with atomics
                (void)hipGetLastError();
                R = 0;
            } else if (rc != FGA_OK) {
                return rc;
            }
        }
        if (R > 0) {
            base = (char *)ctx->det_log;
            A.out = DcOut{dc, (double *)base, (int *)(base + rec_bytes), cap, R, ctx->g.n1,
                          ctx->g.n2};
            A.logcnt = (int *)(base + rec_bytes + cell_bytes);
        }
        hipLaunchKernelGGL(kernel, grid, block, 0, ctx->stream, A);
        FGA_HIP(ctx, hipGetLastError());
        if (R == 0) return FGA_OK;
        // the logged records (every log at most R long; the rest went to dc
        // with atomics) summed by cell in a fixed order, as in the
        // deterministic mode: on this chip it is faster than adding them
        // with FP64 atomics, whose contention where rays cross is high
        int64_t st[3];
        rc = fga_det_stats(ctx, beams, nshots, R, st);
        if (rc != FGA_OK) return rc;
        return fga_det_reduce(ctx, cap, R, st[0], st[1], dc);
    }
    // deterministic: log, check the longest log (rerun with that length if
    // some beam ran past the slots), then reduce in a fixed order.  A rerun
    // must start from the same initial cotangent, so an aliased lam0 is kept.
    if (lam0 && lam0 == lam_out) {
        rc = fga_ensure(ctx, &ctx->det_lam, &ctx->det_lam_bytes,
                        (size_t)FGA_NSTATE * cap * sizeof(double), "initial cotangent copy");
        if (rc != FGA_OK) return rc;
        FGA_HIP(ctx, hipMemcpyAsync(ctx->det_lam, lam0, (size_t)FGA_NSTATE * cap * sizeof(double),
                                    hipMemcpyDeviceToDevice, ctx->stream));
        A.lam0 = (const double *)ctx->det_lam;
    }
    int R = ctx->det_R > 0 ? ctx->det_R : (int)std::min<int64_t>(4 * steps + 1, 64);
    int64_t st[3];
    for (;;) {
        const size_t rec_bytes = (size_t)R * 16 * cap * sizeof(double);
        const size_t cell_bytes = (size_t)R * cap * sizeof(int);
        rc = fga_ensure(ctx, &ctx->det_log, &ctx->det_log_bytes,
                        rec_bytes + cell_bytes + (size_t)cap * sizeof(int), "dJ/dc logs");
        if (rc != FGA_OK) return rc;
        char *base = (char *)ctx->det_log;
        A.out = DcOut{nullptr, (double *)base, (int *)(base + rec_bytes), cap, R, ctx->g.n1,
                      ctx->g.n2};
        A.logcnt = (int *)(base + rec_bytes + cell_bytes);
        hipLaunchKernelGGL(kernel, grid, block, 0, ctx->stream, A);
        FGA_HIP(ctx, hipGetLastError());
        rc = fga_det_stats(ctx, beams, nshots, R, st);
        if (rc != FGA_OK) return rc;
        if (st[2] <= R) break;
        R = (int)st[2];
        ctx->det_R = R;
    }
    return fga_det_reduce(ctx, cap, R, st[0], st[1], dc);
}

// ------------------------------------------------------ reconstruction adjoint
//
// dJ/d(beam) for J = sum_x du(x) u(x), u the recons eq. over the truncation
// boxes (held fixed).  With r = x - Q, the term of a beam is
//   E(x) = C a e^{iS/eps} g1(x1) g2(x2),  g_k = e^{i P_k r_k / eps - r_k^2 / (2 eps)},
// so every derivative of Re E summed against du needs only the three sums
//   F = sum du g1 g2,  F1 = sum du g1 r1 g2,  F2 = sum du g1 g2 r2,
// taken as column sums: a lane owns one x1 of the box and runs down the rows
// (coalesced du loads), g2 and g2 r2 of 256 rows at a time sit in LDS.  Then
// with W = C a e^{iS/eps}:
//   dQ_k = (P_k Im(W F) + Re(W F_k)) / eps,  dP_k = -Im(W F_k) / eps,
//   dS = -Im(W F) / eps,  d(Re a, Im a) = (Re X, -Im X) with X = C e^{iS/eps} F,
//   d(Re C, Im C) = (Re Y, -Im Y) with Y = a e^{iS/eps} F.
// One wavefront per beam; FP64.
#define RA_ROWS 256

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256)
k_reconstruct_adjoint(const double *__restrict__ f, const int64_t *__restrict__ id,
                      const int64_t *__restrict__ offsets, int nshots, int64_t cap, int64_t NqNp,
                      const double *__restrict__ du, int n1, int n2, double o1, double o2,
                      double d1, double d2, double eps, int Rw1, int Rw2,
                      double *__restrict__ dstate, double *__restrict__ dcoef)
{
    __shared__ double2 gv[4][RA_ROWS], gr[4][RA_ROWS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double2 *V = gv[wave], *Vr = gr[wave];
    const int64_t nb = offsets[nshots];
    const double inv_eps = 1.0 / eps, h_inv_eps = 0.5 / eps;
    for (int64_t b = (int64_t)blockIdx.x * 4 + wave; b < nb; b += (int64_t)gridDim.x * 4) {
        const double *st = f + (size_t)FGA_F_STATE * cap + b;
        const double Q1 = st[0], Q2 = st[cap], P1 = st[2 * cap], P2 = st[3 * cap];
        const double S = st[4 * cap];
        const Cd a = {st[21 * cap], st[22 * cap]};
        const Cd C = {f[4 * cap + b], f[5 * cap + b]};
        const int shot = (int)(id[b] / (2 * NqNp));
        const double *dus = du + (size_t)shot * n1 * n2;
        const BeamBox bx = beam_box(Q1, Q2, o1, o2, d1, d2, Rw1, Rw2, n1, n2);
        Cd F = {0.0, 0.0}, F1 = {0.0, 0.0}, F2 = {0.0, 0.0};
        for (int c0 = bx.lo1; c0 <= bx.hi1; c0 += 64) {
            const int x1 = c0 + lane;
            const bool in1 = x1 <= bx.hi1;
            const double r1 = (o1 + x1 * d1) - Q1;
            double sn, cs;
            sincos(P1 * r1 * inv_eps, &sn, &cs);
            const double e1 = exp(-r1 * r1 * h_inv_eps);
            const Cd g1 = {e1 * cs, e1 * sn};
            Cd col = {0.0, 0.0}, colr = {0.0, 0.0};
            for (int r0 = bx.lo2; r0 <= bx.hi2; r0 += RA_ROWS) {
                const int nr = min(RA_ROWS, bx.hi2 - r0 + 1);
                __builtin_amdgcn_wave_barrier();
                for (int i = lane; i < nr; i += 64) {
                    const double r2 = (o2 + (r0 + i) * d2) - Q2;
                    double s2, c2;
                    sincos(P2 * r2 * inv_eps, &s2, &c2);
                    const double e2 = exp(-r2 * r2 * h_inv_eps);
                    V[i] = double2{e2 * c2, e2 * s2};
                    Vr[i] = double2{e2 * c2 * r2, e2 * s2 * r2};
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (in1) {
                    const double *p = dus + (size_t)r0 * n1 + x1;
#pragma unroll 4
                    for (int i = 0; i < nr; ++i) {
                        const double d = p[(size_t)i * n1];
                        const double2 v = V[i], w = Vr[i];
                        col.r = fma(v.x, d, col.r);
                        col.i = fma(v.y, d, col.i);
                        colr.r = fma(w.x, d, colr.r);
                        colr.i = fma(w.y, d, colr.i);
                    }
                }
            }
            if (in1) {
                const Cd t = cmul(g1, col);
                F = cadd(F, t);
                F1 = cadd(F1, cscale(t, r1));
                F2 = cadd(F2, cmul(g1, colr));
            }
        }
        F = {wave_sum(F.r), wave_sum(F.i)};
        F1 = {wave_sum(F1.r), wave_sum(F1.i)};
        F2 = {wave_sum(F2.r), wave_sum(F2.i)};
        if (lane == 0) {
            double sn, cs;
            sincos(S * inv_eps, &sn, &cs);
            const Cd H = {cs, sn};
            const Cd W = cmul(cmul(C, a), H);
            const Cd E = cmul(W, F), E1 = cmul(W, F1), E2 = cmul(W, F2);
            const Cd X = cmul(cmul(C, H), F), Y = cmul(cmul(a, H), F);
            double *o = dstate + b;
            o[0] = (P1 * E.i + E1.r) * inv_eps;
            o[cap] = (P2 * E.i + E2.r) * inv_eps;
            o[2 * cap] = -E1.i * inv_eps;
            o[3 * cap] = -E2.i * inv_eps;
            o[4 * cap] = -E.i * inv_eps;
            for (int k = 5; k < 21; ++k) o[(size_t)k * cap] = 0.0;
            o[21 * cap] = X.r;
            o[22 * cap] = -X.i;
            dcoef[b] = Y.r;
            dcoef[cap + b] = -Y.i;
        }
    }
}

fga_status fga_launch_reconstruct_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                          const double *du, double *dstate, double *dcoef)
{
    const int64_t NqNp = (int64_t)ctx->p.nq1 * ctx->p.nq2 * ctx->p.np1 * ctx->p.np2;
    const fga_grid &g = ctx->g;
    hipLaunchKernelGGL(k_reconstruct_adjoint, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream,
                       beams->f, beams->id, beams->offsets, nshots, beams->capacity, NqNp, du,
                       g.n1, g.n2, g.o1, g.o2, g.d1, g.d2, ctx->p.eps, ctx->Rw1, ctx->Rw2,
                       dstate, dcoef);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

// ------------------------------------------------------- decomposition adjoint

template <typename R>
struct cplxR {
    R re, im;
};

__global__ void k_fill_zero(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// dJ/dpsi_0 (and dJ/dpsi_1, dJ/dc(q)) in the layout of the forward FBI
// output, from dJ/dC of every beam.  psi_{+-} = (psi0 + sigma i r psi1)/2 with
// r = eps / (c(q)|p|); the two branches of one (q, p) add to the same slot
// (two additions to zero commute exactly, so the result is deterministic).
template <typename R>
__global__ void k_scatter_psib(const int64_t *__restrict__ id, const int64_t *__restrict__ offsets,
                               int nshots, const double *__restrict__ gcoef, int64_t cap,
                               const cplxR<R> *__restrict__ Psi, const double *__restrict__ cq,
                               int nq1, int nq2, int np1, int np2, int nfj, double dp1,
                               double dp2, double eps, double norm, double *psib, double *cqb,
                               double *cqc)
{
    const int64_t nb = offsets[nshots];
    const int64_t Nq = (int64_t)nq1 * nq2, Np = (int64_t)np1 * np2, NqNp = Nq * Np;
    const size_t NC = (size_t)nq1 * np1;
    const size_t plane = (size_t)nq2 * np2 * NC;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        int64_t cid = id[b];
        int s = (int)(cid / (2 * NqNp));
        int64_t cl = cid - (int64_t)s * 2 * NqNp;
        int sb = (int)(cl / NqNp);
        int64_t rem = cl - sb * NqNp;
        int64_t qf = rem / Np, pf = rem - qf * Np;
        int j2 = (int)(qf / nq1), j1 = (int)(qf - (int64_t)j2 * nq1);
        int l2 = (int)(pf / np1), l1 = (int)(pf - (int64_t)l2 * np1);
        size_t off = ((size_t)j2 * np2 + l2) * NC + (size_t)j1 * np1 + l1;
        // dJ/dpsi_{+-} = norm dJ/dC
        double pr = norm * gcoef[b], pi = norm * gcoef[cap + b];
        double *p0 = psib + 2 * ((size_t)(s * nfj) * plane + off);
        atomicAdd(p0, 0.5 * pr);
        atomicAdd(p0 + 1, 0.5 * pi);
        if (nfj == 2) {
            double sg = sb == 0 ? 1.0 : -1.0;
            double pp1 = (l1 - 0.5 * (np1 - 1)) * dp1, pp2 = (l2 - 0.5 * (np2 - 1)) * dp2;
            double cqv = cq[qf];
            double r = eps / (cqv * sqrt(pp1 * pp1 + pp2 * pp2));
            // d psi / d psi1 = sigma i r / 2  ->  psi1b += conj(.) psib = -sigma i r/2 psib
            double *p1 = psib + 2 * ((size_t)(s * nfj + 1) * plane + off);
            atomicAdd(p1, 0.5 * sg * r * pi);
            atomicAdd(p1 + 1, -0.5 * sg * r * pr);
            // d psi / d r = sigma i psi1 / 2 ; d r / d c(q) = -r / c(q)
            cplxR<R> v = Psi[(size_t)(s * nfj + 1) * plane + off];
            double wr = -0.5 * sg * (double)v.im, wi = 0.5 * sg * (double)v.re;
            double rb = wr * pr + wi * pi;
            if (cqc)
                cqc[b] = rb * (-r / cqv);
            else
                atomicAdd(&cqb[qf], rb * (-r / cqv));
        }
    }
}

// dc += dJ/dc(q) pulled through the B-spline at every q node
__global__ void k_cq_adjoint(VelGrid V, const double *cqb, double o1, double o2, double d1,
                             double d2, int qb1, int qb2, int qs1, int qs2, int nq1, int nq2,
                             double *dc)
{
    // one thread per node, or (deterministic mode, a 1 x 1 launch) one thread
    // walking the nodes in order, so that the additions come in a fixed order
    const DcOut out = {dc, nullptr, nullptr, 0, 0, V.n1, V.n2};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nq1 * nq2;
         i += gridDim.x * blockDim.x) {
        int j1 = i % nq1, j2 = i / nq1;
        double x1 = o1 + (qb1 + j1 * qs1) * d1, x2 = o2 + (qb2 + j2 * qs2) * d2;
        Vel3 v;
        vel_eval3(V, x1, x2, v);
        double vb[6] = {cqb[i], 0, 0, 0, 0, 0};
        DcAcc dacc;
        dcacc_init(dacc);
        scatter_dc(v, vb, dacc, out);
        dcacc_flush(dacc, out);
    }
}

// Deterministic dJ/dc(q): the per-beam contributions (cqc) summed for every q
// node over the shots and branches in order, each over its beams in id order
// (the beams of one (shot, branch, q) are contiguous: ids sorted ascending).
__global__ void k_cqb_gather(const int64_t *__restrict__ id, const int64_t *__restrict__ offsets,
                             int nshots, const double *__restrict__ cqc, int64_t Nq, int64_t Np,
                             double *cqb)
{
    const int64_t qf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qf >= Nq) return;
    const int64_t nb = offsets[nshots];
    double acc = 0.0;
    for (int s = 0; s < nshots; ++s)
        for (int br = 0; br < 2; ++br) {
            const int64_t lo = ((int64_t)(2 * s + br) * Nq + qf) * Np, hi = lo + Np;
            int64_t a = 0, z = nb;   // first beam with id >= lo
            while (a < z) {
                const int64_t m = (a + z) >> 1;
                if (id[m] < lo) a = m + 1; else z = m;
            }
            for (int64_t b = a; b < nb && id[b] < hi; ++b) acc += cqc[b];
        }
    cqb[qf] = acc;
}

// Transposed pass 2: Tb[sf][i2][c] = d2 sum_{j2, l2} conj(E2[l2][i2 - k2(j2)]) psib[sf][j2][l2][c]
// A thread owns column c of P2T_ROWS consecutive rows i2, so each psib entry
// is loaded once for the rows of the block its window covers (the windows of
// neighbouring rows overlap almost entirely); every output still sums over
// j2, then l2, in increasing order.
#define P2T_ROWS 8

template <typename R>
__global__ void __launch_bounds__(256)
k_fbi_pass2_t(const double *__restrict__ psib, const cplxR<R> *__restrict__ E2, double *Tb,
              int n2, int R2, int qb2, int qs2, int nq2, int np2, int NC, double d2)
{
    const int W2 = 2 * R2 + 1;
    const int i2b = blockIdx.y * P2T_ROWS, sf = blockIdx.z;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NC) return;
    double ar[P2T_ROWS], ai[P2T_ROWS];
#pragma unroll
    for (int r = 0; r < P2T_ROWS; ++r) ar[r] = ai[r] = 0.0;
    for (int j2 = 0; j2 < nq2; ++j2) {
        const int m0 = i2b - (qb2 + j2 * qs2);   // window offset of row i2b from q node j2
        if (m0 + P2T_ROWS - 1 < -R2 || m0 > R2) continue;
        const double *pb = psib + 2 * (((size_t)sf * nq2 + j2) * np2 * (size_t)NC + c);
        for (int l2 = 0; l2 < np2; ++l2) {
            const double br = pb[2 * (size_t)l2 * NC], bi = pb[2 * (size_t)l2 * NC + 1];
            const cplxR<R> *el = E2 + (size_t)l2 * W2 + R2;
#pragma unroll
            for (int r = 0; r < P2T_ROWS; ++r) {
                const int m = m0 + r;
                if (m < -R2 || m > R2) continue;   // uniform in the workgroup
                const cplxR<R> e = el[m];
                const double er = (double)e.re, ei = (double)e.im;
                // conj(e) * b
                ar[r] += er * br + ei * bi;
                ai[r] += er * bi - ei * br;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < P2T_ROWS; ++r) {
        if (i2b + r >= n2) break;
        double *out = Tb + 2 * (((size_t)sf * n2 + i2b + r) * NC + c);
        out[0] = ar[r] * d2;
        out[1] = ai[r] * d2;
    }
}

// the pass-1 table with the window offset fastest: E1tt[l][m] = E1t[m][l]
template <typename R>
__global__ void k_e1_transpose(const cplxR<R> *__restrict__ E1t, cplxR<R> *__restrict__ E1tt,
                               int W1, int np1)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < W1 * np1;
         i += gridDim.x * blockDim.x) {
        const int m = i / np1, l = i - m * np1;
        E1tt[(size_t)l * W1 + m] = E1t[i];
    }
}

// Transposed pass 1: fb[sf][i2][i1] = d1 Re sum_{j1, l1} conj(E1t[i1 - k1(j1)][l1]) Tb[sf][i2][j1 np1 + l1]
// (the table read as E1tt[l1][m]: neighbouring lanes, neighbouring m)
template <typename R>
__global__ void __launch_bounds__(256)
k_fbi_pass1_t(const double *__restrict__ Tb, const cplxR<R> *__restrict__ E1tt, double *f0b,
              double *f1b, int nfj, int n1, int n2, int R1, int qb1, int qs1, int nq1, int np1,
              double d1)
{
    const int i1 = blockIdx.x * blockDim.x + threadIdx.x;
    const int i2 = blockIdx.y, sf = blockIdx.z;
    if (i1 >= n1) return;
    const int NC = nq1 * np1, W1 = 2 * R1 + 1;
    const double *tb = Tb + 2 * (((size_t)sf * n2 + i2) * NC);
    double acc = 0.0;
    for (int j1 = 0; j1 < nq1; ++j1) {
        const int m = i1 - (qb1 + j1 * qs1);   // window offset of node i1 from q node j1
        if (m < -R1 || m > R1) continue;
        const cplxR<R> *e = E1tt + (m + R1);
        const double *t = tb + 2 * (size_t)j1 * np1;
        for (int l1 = 0; l1 < np1; ++l1) {
            // Re(conj(e) t)
            const cplxR<R> v = e[(size_t)l1 * W1];
            acc += (double)v.re * t[2 * l1] + (double)v.im * t[2 * l1 + 1];
        }
    }
    int s = sf / nfj, fj = sf % nfj;
    double *out = fj == 0 ? f0b : f1b;
    if (out) out[((size_t)s * n2 + i2) * n1 + i1] = acc * d1;
}

template <typename R>
static fga_status decompose_adjoint_impl(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                         const double *gcoef, double *df0, double *df1,
                                         double *dc)
{
    const fga_grid &g = ctx->g;
    const fga_params &p = ctx->p;
    hipStream_t st = ctx->stream;
    const int nfj = ctx->last_nfj;
    const int S = nshots * nfj;
    const size_t NC = (size_t)p.nq1 * p.np1;
    const size_t psib_elems = (size_t)S * p.nq2 * p.np2 * NC * 2;
    const size_t tb_elems = (size_t)S * g.n2 * NC * 2;
    fga_status rc = fga_ensure(ctx, &ctx->adj_psib, &ctx->adj_psib_bytes,
                               (psib_elems + tb_elems + (size_t)p.nq1 * p.nq2) * sizeof(double),
                               "decomposition adjoint workspace");
    if (rc != FGA_OK) return rc;
    const bool det = ctx->p.deterministic && nfj == 2 && dc;
    if (det) {
        rc = fga_ensure(ctx, &ctx->det_cqc, &ctx->det_cqc_bytes,
                        (size_t)beams->capacity * sizeof(double), "c(q) cotangents");
        if (rc != FGA_OK) return rc;
    }
    double *psib = (double *)ctx->adj_psib;
    double *Tb = psib + psib_elems;
    double *cqb = Tb + tb_elems;
    hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, st, psib,
                       (int64_t)(psib_elems + tb_elems + (size_t)p.nq1 * p.nq2));
    hipLaunchKernelGGL(k_scatter_psib<R>, dim3(ctx->num_cu * 4), dim3(256), 0, st, beams->id,
                       beams->offsets, nshots, gcoef, beams->capacity,
                       (const cplxR<R> *)ctx->Psi, ctx->cq, p.nq1, p.nq2, p.np1, p.np2, nfj,
                       p.dp1, p.dp2, p.eps, ctx->norm, psib, cqb,
                       det ? (double *)ctx->det_cqc : nullptr);
    hipLaunchKernelGGL(k_fbi_pass2_t<R>,
                       dim3((unsigned)((NC + 255) / 256), (g.n2 + P2T_ROWS - 1) / P2T_ROWS, S),
                       dim3(256),
                       0, st, psib, (const cplxR<R> *)ctx->E2, Tb, g.n2, ctx->R2, p.qb2, p.qs2,
                       p.nq2, p.np2, (int)NC, g.d2);
    const int W1 = 2 * ctx->R1 + 1;
    rc = fga_ensure(ctx, &ctx->E1tt, &ctx->E1tt_bytes, (size_t)W1 * p.np1 * sizeof(cplxR<R>),
                    "transposed pass-1 table");
    if (rc != FGA_OK) return rc;
    hipLaunchKernelGGL(k_e1_transpose<R>, dim3((W1 * p.np1 + 255) / 256), dim3(256), 0, st,
                       (const cplxR<R> *)ctx->E1t, (cplxR<R> *)ctx->E1tt, W1, p.np1);
    hipLaunchKernelGGL(k_fbi_pass1_t<R>, dim3((g.n1 + 255) / 256, g.n2, S), dim3(256), 0, st, Tb,
                       (const cplxR<R> *)ctx->E1tt, df0, df1, nfj, g.n1, g.n2, ctx->R1, p.qb1,
                       p.qs1, p.nq1, p.np1, g.d1);
    if (nfj == 2 && dc) {
        int nq = p.nq1 * p.nq2;
        if (det)
            hipLaunchKernelGGL(k_cqb_gather, dim3((nq + 255) / 256), dim3(256), 0, st, beams->id,
                               beams->offsets, nshots, (const double *)ctx->det_cqc, (int64_t)nq,
                               (int64_t)p.np1 * p.np2, cqb);
        hipLaunchKernelGGL(k_cq_adjoint, det ? dim3(1) : dim3((nq + 255) / 256),
                           det ? dim3(1) : dim3(256), 0, st,
                           fga_velgrid(ctx), cqb, g.o1, g.o2, g.d1, g.d2, p.qb1, p.qb2, p.qs1,
                           p.qs2, p.nq1, p.nq2, dc);
    }
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}

fga_status fga_launch_decompose_adjoint(fga_ctx *ctx, const fga_beams *beams, int nshots,
                                        const double *gcoef, double *df0, double *df1, double *dc)
{
    if (ctx->prec == FGA_FP64)
        return decompose_adjoint_impl<double>(ctx, beams, nshots, gcoef, df0, df1, dc);
    return decompose_adjoint_impl<float>(ctx, beams, nshots, gcoef, df0, df1, dc);
}
