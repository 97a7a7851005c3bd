/*
 * Plain FP64 CPU oracle of the frozen Gaussian approximation (FGA) for the
 * 2-D acoustic wave equation u_tt = c(x)^2 Lap u (Yang, Lu and Fomel,
 * "Seismic modeling using the frozen Gaussian approximation").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code with the
 * HIP path.  Everything is a direct loop in double precision, following the
 * paper's steps in its own order and notation; nothing is blocked, fused or
 * factorised beyond what the equations state.
 *
 * Conventions (readings of points the paper leaves open):
 *   - grid nodes x_i = o + i*d, arrays C-ordered [n2][n1];
 *   - c(x) is the uniform cubic B-spline with the grid samples as
 *     coefficients, indices clamped to the grid (the paper does not say how
 *     c is represented; the dynamic ray tracing equations need second
 *     derivatives of c, so the interpolant must be C^2);
 *   - the FBI integral is a Riemann sum on the grid nodes with weight d1*d2,
 *     f = 0 outside the grid, truncated to the box |m_i d_i| <= R_i d_i with
 *     R_i = ceil(sqrt(2 eps ln(1/tau_fbi)) / d_i) (the paper's box B_eps of
 *     side O(sqrt(eps)));
 *   - the sum over (q,p) in the reconstruction is a phase-space quadrature
 *     with weight w = (qs1 d1)(qs2 d2) dp1 dp2;
 *   - the reconstruction sum is truncated to the square box of half-width
 *     Rw_i = ceil(sqrt(2 eps ln(1/tau_win)) / d_i) around the node nearest Q,
 *     clipped to the grid.
 *
 * Beam state (23 doubles per beam, AoS):
 *   0 Q1, 1 Q2, 2 P1, 3 P2, 4 S,
 *   5..12  A = dz Q  (complex 2x2, row-major, re/im interleaved),
 *   13..20 B = dz P  (same layout),
 *   21 a_re, 22 a_im.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NSTATE 23

/* ------------------------------------------------------------------ */
/* Uniform cubic B-spline and its derivatives (velocity interpolant)   */
/* ------------------------------------------------------------------ */

/* beta3(s) and its first three derivatives in s.  The third derivative is
 * piecewise constant; at a knot the right-hand value is taken. */
static double beta3(double s, int deriv)
{
    double a = fabs(s);
    double sg = (s < 0.0) ? -1.0 : 1.0;
    if (a < 1.0) {
        switch (deriv) {
        case 0: return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        case 1: return sg * (-2.0 * a + 1.5 * a * a);
        case 2: return -2.0 + 3.0 * a;
        default: return (s < 0.0) ? -3.0 : 3.0;
        }
    }
    if (a < 2.0) {
        double b = 2.0 - a;
        switch (deriv) {
        case 0: return b * b * b / 6.0;
        case 1: return -sg * 0.5 * b * b;
        case 2: return b;
        default: return (s < 0.0) ? 1.0 : -1.0;
        }
    }
    return 0.0;
}

static int clampi(int k, int n)
{
    return k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
}

/* c and its partial derivatives at (x1, x2); the first nout entries of
 * out = {c, c_1, c_2, c_11, c_12, c_22, c_111, c_112, c_122, c_222}.
 * beta3(t - k) vanishes unless |t - k| < 2, i.e. k = floor(t)-1 .. floor(t)+2,
 * so those four knots per axis carry the whole sum. */
static void velocity_n(const double *c, int n1, int n2, double o1, double o2,
                       double d1, double d2, double x1, double x2, int nout,
                       double *out)
{
    static const int D1[10] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0};
    static const int D2[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};
    double t1 = (x1 - o1) / d1, t2 = (x2 - o2) / d2;
    int i1 = (int)floor(t1), i2 = (int)floor(t2);
    double w1[4][4], w2[4][4];  /* [derivative order][knot] */
    for (int dd = 0; dd < 4; ++dd)
        for (int k = 0; k < 4; ++k) {
            w1[dd][k] = beta3(t1 - (i1 - 1 + k), dd) / pow(d1, dd);
            w2[dd][k] = beta3(t2 - (i2 - 1 + k), dd) / pow(d2, dd);
        }
    for (int r = 0; r < nout; ++r) out[r] = 0.0;
    for (int k2 = 0; k2 < 4; ++k2) {
        for (int k1 = 0; k1 < 4; ++k1) {
            double ck = c[(size_t)clampi(i2 - 1 + k2, n2) * n1 + clampi(i1 - 1 + k1, n1)];
            for (int r = 0; r < nout; ++r)
                out[r] += ck * w1[D1[r]][k1] * w2[D2[r]][k2];
        }
    }
}

void or_velocity(const double *c, int n1, int n2, double o1, double o2,
                 double d1, double d2, double x1, double x2, double *out)
{
    velocity_n(c, n1, n2, o1, o2, d1, d2, x1, x2, 10, out);
}

void or_velocity_points(const double *c, int n1, int n2, double o1, double o2,
                        double d1, double d2, int64_t npts, const double *x1,
                        const double *x2, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i)
        or_velocity(c, n1, n2, o1, o2, d1, d2, x1[i], x2[i], out + 10 * i);
}

/* ------------------------------------------------------------------ */
/* Step 1: FBI transform (psi eq.) with the local box B_eps            */
/* ------------------------------------------------------------------ */

static int window_halfwidth(double eps, double tau, double d)
{
    return (int)ceil(sqrt(2.0 * eps * log(1.0 / tau)) / d);
}

static double pmesh(int l, int np, double dp)
{
    return (l - 0.5 * (np - 1)) * dp;
}

/* First and last column of every row where f is nonzero (lo > hi for a row
 * of zeros).  A term with f = 0 adds exactly zero to the sums below, so the
 * loops may pass over those columns without changing any result. */
static void row_support(const double *f, int n1, int n2, int *lo, int *hi)
{
    for (int y2 = 0; y2 < n2; ++y2) {
        const double *row = f + (size_t)y2 * n1;
        int a = 0, b = n1 - 1;
        while (a < n1 && row[a] == 0.0) ++a;
        while (b >= a && row[b] == 0.0) --b;
        lo[y2] = a;
        hi[y2] = b;
    }
}

/* psi_j(q,p) = d1 d2 sum_m f(k+m) exp(-|m d|^2/(2 eps)) exp(-i p.(m d)/eps)
 * for every q node k = (qb1 + j1 qs1, qb2 + j2 qs2) and p-mesh node.
 * Output: psi[(((j2*nq1 + j1)*np2 + l2)*np1 + l1)*2 + {0: re, 1: im}].
 * The one-dimensional factors of the kernel are tabulated once; each
 * (q, p) pair is then a direct double sum over the box (terms where f
 * vanishes are passed over: they add exactly zero). */
void or_fbi(const double *f, int n1, int n2, double d1, double d2, double eps,
            double tau_fbi, int qb1, int qb2, int qs1, int qs2, int nq1,
            int nq2, int np1, int np2, double dp1, double dp2, double *psi)
{
    int R1 = window_halfwidth(eps, tau_fbi, d1);
    int R2 = window_halfwidth(eps, tau_fbi, d2);
    int W1 = 2 * R1 + 1, W2 = 2 * R2 + 1;
    double complex *E1 = malloc(sizeof(double complex) * (size_t)np1 * W1);
    double complex *E2 = malloc(sizeof(double complex) * (size_t)np2 * W2);
    for (int l = 0; l < np1; ++l)
        for (int m = -R1; m <= R1; ++m) {
            double r = m * d1;
            E1[(size_t)l * W1 + m + R1] =
                exp(-r * r / (2.0 * eps)) * cexp(-I * pmesh(l, np1, dp1) * r / eps);
        }
    for (int l = 0; l < np2; ++l)
        for (int m = -R2; m <= R2; ++m) {
            double r = m * d2;
            E2[(size_t)l * W2 + m + R2] =
                exp(-r * r / (2.0 * eps)) * cexp(-I * pmesh(l, np2, dp2) * r / eps);
        }
    int *lo = malloc(sizeof(int) * (size_t)n2), *hi = malloc(sizeof(int) * (size_t)n2);
    row_support(f, n1, n2, lo, hi);
    int64_t nq = (int64_t)nq1 * nq2, np = (int64_t)np1 * np2;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int64_t jq = 0; jq < nq; ++jq) {
        for (int64_t lp = 0; lp < np; ++lp) {
            int j1 = (int)(jq % nq1), j2 = (int)(jq / nq1);
            int l1 = (int)(lp % np1), l2 = (int)(lp / np1);
            int k1 = qb1 + j1 * qs1, k2 = qb2 + j2 * qs2;
            const double complex *e1 = E1 + (size_t)l1 * W1;
            const double complex *e2 = E2 + (size_t)l2 * W2;
            double complex acc = 0.0;
            for (int m2 = -R2; m2 <= R2; ++m2) {
                int y2 = k2 + m2;
                if (y2 < 0 || y2 >= n2 || lo[y2] > hi[y2]) continue;
                const double *row = f + (size_t)y2 * n1;
                int m1a = lo[y2] - k1 > -R1 ? lo[y2] - k1 : -R1;
                int m1b = hi[y2] - k1 < R1 ? hi[y2] - k1 : R1;
                if (m1a > m1b) continue;
                double sr = 0.0, si = 0.0;
                for (int m1 = m1a; m1 <= m1b; ++m1) {
                    int y1 = k1 + m1;
                    sr += row[y1] * creal(e1[m1 + R1]);
                    si += row[y1] * cimag(e1[m1 + R1]);
                }
                acc += e2[m2 + R2] * (sr + I * si);
            }
            acc *= d1 * d2;
            psi[(jq * np + lp) * 2 + 0] = creal(acc);
            psi[(jq * np + lp) * 2 + 1] = cimag(acc);
        }
    }
    free(E1);
    free(E2);
    free(lo);
    free(hi);
}

/* A bound of |psi_j(q,p)| that holds for every p at each q node:
 * bound(q) = d1 d2 sum_m |f(k+m)| exp(-|m d|^2/(2 eps)) over the same box
 * (the modulus of a sum is at most the sum of the moduli, and the Fourier
 * factor has modulus 1).  Output bound[j2*nq1 + j1]. */
void or_fbi_bound(const double *f, int n1, int n2, double d1, double d2, double eps,
                  double tau_fbi, int qb1, int qb2, int qs1, int qs2, int nq1, int nq2,
                  double *bound)
{
    int R1 = window_halfwidth(eps, tau_fbi, d1);
    int R2 = window_halfwidth(eps, tau_fbi, d2);
    double *w1 = malloc(sizeof(double) * (size_t)(2 * R1 + 1));
    double *w2 = malloc(sizeof(double) * (size_t)(2 * R2 + 1));
    for (int m = -R1; m <= R1; ++m) w1[m + R1] = exp(-(m * d1) * (m * d1) / (2.0 * eps));
    for (int m = -R2; m <= R2; ++m) w2[m + R2] = exp(-(m * d2) * (m * d2) / (2.0 * eps));
    int *lo = malloc(sizeof(int) * (size_t)n2), *hi = malloc(sizeof(int) * (size_t)n2);
    row_support(f, n1, n2, lo, hi);
    int64_t nq = (int64_t)nq1 * nq2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t jq = 0; jq < nq; ++jq) {
        int k1 = qb1 + (int)(jq % nq1) * qs1, k2 = qb2 + (int)(jq / nq1) * qs2;
        double acc = 0.0;
        for (int m2 = -R2; m2 <= R2; ++m2) {
            int y2 = k2 + m2;
            if (y2 < 0 || y2 >= n2 || lo[y2] > hi[y2]) continue;
            const double *row = f + (size_t)y2 * n1;
            double s = 0.0;
            for (int m1 = -R1; m1 <= R1; ++m1) {
                int y1 = k1 + m1;
                if (y1 < 0 || y1 >= n1) continue;
                s += fabs(row[y1]) * w1[m1 + R1];
            }
            acc += w2[m2 + R2] * s;
        }
        bound[jq] = d1 * d2 * acc;
    }
    free(w1);
    free(w2);
    free(lo);
    free(hi);
}

/* ------------------------------------------------------------------ */
/* Step 2: ray tracing, dynamic ray tracing and amplitude (RK4)        */
/* ------------------------------------------------------------------ */

typedef struct {
    const double *c;
    int n1, n2;
    double o1, o2, d1, d2;
} vel_t;

/* Right-hand side of the characteristic equations, the dynamic ray tracing
 * equations for dzQ and dzP, the action and the amplitude equation for the
 * Hamiltonian H = sigma c(Q) |P|. */
static void rhs(const vel_t *v, double sigma, const double *y, double *dy)
{
    double cv[6];
    velocity_n(v->c, v->n1, v->n2, v->o1, v->o2, v->d1, v->d2, y[0], y[1], 6, cv);
    double c = cv[0];
    double g[2] = {cv[1], cv[2]};
    double K[2][2] = {{cv[3], cv[4]}, {cv[4], cv[5]}};
    double P[2] = {y[2], y[3]};
    double n = sqrt(P[0] * P[0] + P[1] * P[1]);
    double u[2] = {P[0] / n, P[1] / n};

    double H = sigma * c * n;
    double HP[2], HQ[2], HPP[2][2], HQQ[2][2], HQP[2][2], HPQ[2][2];
    for (int l = 0; l < 2; ++l) {
        HP[l] = sigma * c * u[l];
        HQ[l] = sigma * n * g[l];
        for (int k = 0; k < 2; ++k) {
            HPP[l][k] = sigma * (c / n) * ((l == k ? 1.0 : 0.0) - u[l] * u[k]);
            HQQ[l][k] = sigma * n * K[l][k];
            HQP[l][k] = sigma * g[l] * u[k];   /* d2H / dQ_l dP_k */
            HPQ[l][k] = sigma * u[l] * g[k];   /* d2H / dP_l dQ_k */
        }
    }

    dy[0] = HP[0];
    dy[1] = HP[1];
    dy[2] = -HQ[0];
    dy[3] = -HQ[1];
    dy[4] = P[0] * HP[0] + P[1] * HP[1] - H;

    double complex A[2][2], B[2][2], dA[2][2], dB[2][2];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
            A[j][k] = y[5 + 2 * (2 * j + k)] + I * y[6 + 2 * (2 * j + k)];
            B[j][k] = y[13 + 2 * (2 * j + k)] + I * y[14 + 2 * (2 * j + k)];
        }
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
            double complex sa = 0.0, sb = 0.0;
            for (int l = 0; l < 2; ++l) {
                sa += A[j][l] * HQP[l][k] + B[j][l] * HPP[l][k];
                sb += -A[j][l] * HQQ[l][k] - B[j][l] * HPQ[l][k];
            }
            dA[j][k] = sa;
            dB[j][k] = sb;
            dy[5 + 2 * (2 * j + k)] = creal(sa);
            dy[6 + 2 * (2 * j + k)] = cimag(sa);
            dy[13 + 2 * (2 * j + k)] = creal(sb);
            dy[14 + 2 * (2 * j + k)] = cimag(sb);
        }

    /* Z = dz(Q + iP) = A + iB; tr(Z^{-1} dZ/dt) with the 2x2 inverse */
    double complex Z[2][2], dZ[2][2], Zi[2][2];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
            Z[j][k] = A[j][k] + I * B[j][k];
            dZ[j][k] = dA[j][k] + I * dB[j][k];
        }
    double complex det = Z[0][0] * Z[1][1] - Z[0][1] * Z[1][0];
    Zi[0][0] = Z[1][1] / det;
    Zi[0][1] = -Z[0][1] / det;
    Zi[1][0] = -Z[1][0] / det;
    Zi[1][1] = Z[0][0] / det;
    double complex tr = 0.0;
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) tr += Zi[j][k] * dZ[k][j];

    double complex a = y[21] + I * y[22];
    double complex da = a * (HP[0] * HQ[0] + HP[1] * HQ[1]) / H + 0.5 * a * tr;
    dy[21] = creal(da);
    dy[22] = cimag(da);
}

/* Classical fourth-order Runge-Kutta, fixed step dt, nsteps steps, for
 * every beam independently.  state: [nb][23]; sigma: [nb] (+1 or -1). */
void or_propagate(const double *c, int n1, int n2, double o1, double o2,
                  double d1, double d2, int64_t nb, const int8_t *sigma,
                  double *state, double dt, int nsteps)
{
    vel_t v = {c, n1, n2, o1, o2, d1, d2};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        double *y = state + (size_t)b * NSTATE;
        double s = (double)sigma[b];
        double k1[NSTATE], k2[NSTATE], k3[NSTATE], k4[NSTATE], t[NSTATE];
        for (int it = 0; it < nsteps; ++it) {
            rhs(&v, s, y, k1);
            for (int i = 0; i < NSTATE; ++i) t[i] = y[i] + 0.5 * dt * k1[i];
            rhs(&v, s, t, k2);
            for (int i = 0; i < NSTATE; ++i) t[i] = y[i] + 0.5 * dt * k2[i];
            rhs(&v, s, t, k3);
            for (int i = 0; i < NSTATE; ++i) t[i] = y[i] + dt * k3[i];
            rhs(&v, s, t, k4);
            for (int i = 0; i < NSTATE; ++i)
                y[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        }
    }
}

/* The same RK4 for every state but the amplitude, which is instead set after
 * every step from the conserved quantity a^2 / (c(Q)^2 det Z) (the closed
 * form that follows the amplitude equation in the paper):
 *   a = c(Q) / c(q) (det Z)^{1/2},  Z = A + iB,
 * taking the square root nearest the previous step's, so that it varies
 * continuously in time.  q: [nb][2] the beams' mesh nodes; the root at the
 * start is recovered from the incoming a (2 at t = 0). */
void or_propagate_closed(const double *c, int n1, int n2, double o1, double o2,
                         double d1, double d2, int64_t nb, const int8_t *sigma,
                         const double *q, double *state, double dt, int nsteps)
{
    vel_t v = {c, n1, n2, o1, o2, d1, d2};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        double *y = state + (size_t)b * NSTATE;
        double s = (double)sigma[b];
        double k1[NSTATE], k2[NSTATE], k3[NSTATE], k4[NSTATE], t[NSTATE];
        double cv[6];
        velocity_n(c, n1, n2, o1, o2, d1, d2, q[2 * b], q[2 * b + 1], 1, cv);
        const double cq = cv[0];
        velocity_n(c, n1, n2, o1, o2, d1, d2, y[0], y[1], 1, cv);
        double complex root = (y[21] + I * y[22]) * cq / cv[0];
        for (int it = 0; it < nsteps; ++it) {
            rhs(&v, s, y, k1);
            for (int i = 0; i < NSTATE; ++i) t[i] = y[i] + 0.5 * dt * k1[i];
            rhs(&v, s, t, k2);
            for (int i = 0; i < NSTATE; ++i) t[i] = y[i] + 0.5 * dt * k2[i];
            rhs(&v, s, t, k3);
            for (int i = 0; i < NSTATE; ++i) t[i] = y[i] + dt * k3[i];
            rhs(&v, s, t, k4);
            for (int i = 0; i < NSTATE; ++i)
                y[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
            double complex Z[2][2];
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k)
                    Z[j][k] = (y[5 + 2 * (2 * j + k)] + I * y[6 + 2 * (2 * j + k)]) +
                              I * (y[13 + 2 * (2 * j + k)] + I * y[14 + 2 * (2 * j + k)]);
            double complex r = csqrt(Z[0][0] * Z[1][1] - Z[0][1] * Z[1][0]);
            if (creal(r * conj(root)) < 0.0) r = -r;
            root = r;
            velocity_n(c, n1, n2, o1, o2, d1, d2, y[0], y[1], 1, cv);
            double complex a = cv[0] / cq * r;
            y[21] = creal(a);
            y[22] = cimag(a);
        }
    }
}

/* Right-hand side of the characteristic equations and the action alone (the
 * rays, for the divided-difference mode): y = {Q1, Q2, P1, P2, S}. */
static void ray_rhs(const vel_t *v, double sigma, const double *y, double *dy)
{
    double cv[3];
    velocity_n(v->c, v->n1, v->n2, v->o1, v->o2, v->d1, v->d2, y[0], y[1], 3, cv);
    double n = sqrt(y[2] * y[2] + y[3] * y[3]);
    double H = sigma * cv[0] * n;
    double HP[2] = {sigma * cv[0] * y[2] / n, sigma * cv[0] * y[3] / n};
    dy[0] = HP[0];
    dy[1] = HP[1];
    dy[2] = -sigma * n * cv[1];
    dy[3] = -sigma * n * cv[2];
    dy[4] = y[2] * HP[0] + y[3] * HP[1] - H;
}

/* dzQ and dzP by divided differences instead of the dynamic ray tracing
 * equations (the alternative the paper names next to the dzQ, dzP eqs.):
 * besides its own ray every beam advances the rays of its eight neighbouring
 * mesh nodes, (q +- h[j] e_j, p) and (q, p +- h[2+j] e_j), j = 1, 2, by the
 * same RK4; after every step
 *   dq_j Q_k = (Q_k(+q_j) - Q_k(-q_j)) / (2 h[j]),
 *   dp_j Q_k = (Q_k(+p_j) - Q_k(-p_j)) / (2 h[2+j]),
 * (likewise for P), A[j][k] = dq_j Q_k - i dp_j Q_k, B[j][k] = dq_j P_k -
 * i dp_j P_k, and a = c(Q)/c(q) (det Z)^{1/2}, Z = A + iB, with the root
 * nearest the previous step's (as in or_propagate_closed).  The neighbouring
 * rays start from the incoming state along its A and B (dq_j Q = Re A[j],
 * dp_j Q = -Im A[j], dq_j P = Re B[j], dp_j P = -Im B[j]): at t = 0 (A = I,
 * B = -iI) they are exactly the rays of the neighbouring mesh nodes. */
void or_propagate_dd(const double *c, int n1, int n2, double o1, double o2,
                     double d1, double d2, int64_t nb, const int8_t *sigma,
                     const double *q, double *state, double dt, int nsteps,
                     const double *h)
{
    vel_t v = {c, n1, n2, o1, o2, d1, d2};
    if (nsteps <= 0) return;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        double *y = state + (size_t)b * NSTATE;
        double s = (double)sigma[b];
        /* ray 0: the beam; 1 + 2j / 2 + 2j: +- q_j; 5 + 2j / 6 + 2j: +- p_j */
        double ray[9][5];
        for (int i = 0; i < 5; ++i) ray[0][i] = y[i];
        for (int m = 0; m < 4; ++m) {
            int j = m & 1, alongp = m >= 2;
            for (int side = 0; side < 2; ++side) {
                double *r = ray[1 + 2 * m + side];
                double sh = (side == 0 ? 1.0 : -1.0) * h[m];
                for (int k = 0; k < 2; ++k) {
                    double dQ = alongp ? -y[6 + 2 * (2 * j + k)] : y[5 + 2 * (2 * j + k)];
                    double dP = alongp ? -y[14 + 2 * (2 * j + k)] : y[13 + 2 * (2 * j + k)];
                    r[k] = y[k] + sh * dQ;
                    r[2 + k] = y[2 + k] + sh * dP;
                }
                r[4] = y[4];
            }
        }
        double cv[3];
        velocity_n(c, n1, n2, o1, o2, d1, d2, q[2 * b], q[2 * b + 1], 1, cv);
        const double cq = cv[0];
        velocity_n(c, n1, n2, o1, o2, d1, d2, y[0], y[1], 1, cv);
        double complex root = (y[21] + I * y[22]) * cq / cv[0];
        for (int it = 0; it < nsteps; ++it) {
            for (int r = 0; r < 9; ++r) {
                double *x = ray[r];
                double k1[5], k2[5], k3[5], k4[5], t[5];
                ray_rhs(&v, s, x, k1);
                for (int i = 0; i < 5; ++i) t[i] = x[i] + 0.5 * dt * k1[i];
                ray_rhs(&v, s, t, k2);
                for (int i = 0; i < 5; ++i) t[i] = x[i] + 0.5 * dt * k2[i];
                ray_rhs(&v, s, t, k3);
                for (int i = 0; i < 5; ++i) t[i] = x[i] + dt * k3[i];
                ray_rhs(&v, s, t, k4);
                for (int i = 0; i < 5; ++i)
                    x[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
            }
            double complex A[2][2], B[2][2], Z[2][2];
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k) {
                    double dqQ = (ray[1 + 2 * j][k] - ray[2 + 2 * j][k]) / (2.0 * h[j]);
                    double dpQ = (ray[5 + 2 * j][k] - ray[6 + 2 * j][k]) / (2.0 * h[2 + j]);
                    double dqP = (ray[1 + 2 * j][2 + k] - ray[2 + 2 * j][2 + k]) / (2.0 * h[j]);
                    double dpP = (ray[5 + 2 * j][2 + k] - ray[6 + 2 * j][2 + k]) / (2.0 * h[2 + j]);
                    A[j][k] = dqQ - I * dpQ;
                    B[j][k] = dqP - I * dpP;
                    Z[j][k] = A[j][k] + I * B[j][k];
                }
            double complex r = csqrt(Z[0][0] * Z[1][1] - Z[0][1] * Z[1][0]);
            if (creal(r * conj(root)) < 0.0) r = -r;
            root = r;
            for (int i = 0; i < 5; ++i) y[i] = ray[0][i];
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k) {
                    y[5 + 2 * (2 * j + k)] = creal(A[j][k]);
                    y[6 + 2 * (2 * j + k)] = cimag(A[j][k]);
                    y[13 + 2 * (2 * j + k)] = creal(B[j][k]);
                    y[14 + 2 * (2 * j + k)] = cimag(B[j][k]);
                }
            velocity_n(c, n1, n2, o1, o2, d1, d2, y[0], y[1], 1, cv);
            double complex a = cv[0] / cq * r;
            y[21] = creal(a);
            y[22] = cimag(a);
        }
    }
}

/* The right-hand side alone, for tests of the equations themselves. */
void or_rhs(const double *c, int n1, int n2, double o1, double o2, double d1,
            double d2, double sigma, const double *y, double *dy)
{
    vel_t v = {c, n1, n2, o1, o2, d1, d2};
    rhs(&v, sigma, y, dy);
}

/* ------------------------------------------------------------------ */
/* Step 3: reconstruction (recons eq.)                                 */
/* ------------------------------------------------------------------ */

/* Contribution of one beam at node (i1, i2):
 * C a exp(i S/eps) exp(i P.(x-Q)/eps - |x-Q|^2/(2 eps)). */
static double complex beam_term(const double *coef, const double *y, double eps,
                                double x1, double x2)
{
    double r1 = x1 - y[0], r2 = x2 - y[1];
    double complex C = coef[0] + I * coef[1];
    double complex a = y[21] + I * y[22];
    double phase = (y[4] + y[2] * r1 + y[3] * r2) / eps;
    double gauss = -(r1 * r1 + r2 * r2) / (2.0 * eps);
    return C * a * cexp(I * phase + gauss);
}

static void beam_box(const double *y, int n1, int n2, double o1, double o2,
                     double d1, double d2, int Rw1, int Rw2, int *lo1, int *hi1,
                     int *lo2, int *hi2)
{
    int c1 = (int)floor((y[0] - o1) / d1 + 0.5);
    int c2 = (int)floor((y[1] - o2) / d2 + 0.5);
    *lo1 = c1 - Rw1 < 0 ? 0 : c1 - Rw1;
    *hi1 = c1 + Rw1 > n1 - 1 ? n1 - 1 : c1 + Rw1;
    *lo2 = c2 - Rw2 < 0 ? 0 : c2 - Rw2;
    *hi2 = c2 + Rw2 > n2 - 1 ? n2 - 1 : c2 + Rw2;
}

/* u[i2][i1] = sum over beams whose box holds the node.  u_im may be NULL. */
void or_reconstruct(int n1, int n2, double o1, double o2, double d1, double d2,
                    double eps, double tau_win, int64_t nb, const double *coef,
                    const double *state, double *u_re, double *u_im)
{
    int Rw1 = window_halfwidth(eps, tau_win, d1);
    int Rw2 = window_halfwidth(eps, tau_win, d2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i2 = 0; i2 < n2; ++i2) {
        double x2 = o2 + i2 * d2;
        for (int i1 = 0; i1 < n1; ++i1) {
            u_re[(size_t)i2 * n1 + i1] = 0.0;
            if (u_im) u_im[(size_t)i2 * n1 + i1] = 0.0;
        }
        for (int64_t b = 0; b < nb; ++b) {
            const double *y = state + (size_t)b * NSTATE;
            int lo1, hi1, lo2, hi2;
            beam_box(y, n1, n2, o1, o2, d1, d2, Rw1, Rw2, &lo1, &hi1, &lo2, &hi2);
            if (i2 < lo2 || i2 > hi2) continue;
            for (int i1 = lo1; i1 <= hi1; ++i1) {
                double complex t = beam_term(coef + 2 * b, y, eps, o1 + i1 * d1, x2);
                u_re[(size_t)i2 * n1 + i1] += creal(t);
                if (u_im) u_im[(size_t)i2 * n1 + i1] += cimag(t);
            }
        }
    }
}

/* The same sum at a list of nodes (flat index i2*n1 + i1). */
void or_reconstruct_points(int n1, int n2, double o1, double o2, double d1,
                           double d2, double eps, double tau_win, int64_t nb,
                           const double *coef, const double *state,
                           int64_t npts, const int64_t *nodes, double *out_re,
                           double *out_im)
{
    int Rw1 = window_halfwidth(eps, tau_win, d1);
    int Rw2 = window_halfwidth(eps, tau_win, d2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < npts; ++k) {
        int i1 = (int)(nodes[k] % n1), i2 = (int)(nodes[k] / n1);
        double complex acc = 0.0;
        for (int64_t b = 0; b < nb; ++b) {
            const double *y = state + (size_t)b * NSTATE;
            int lo1, hi1, lo2, hi2;
            beam_box(y, n1, n2, o1, o2, d1, d2, Rw1, Rw2, &lo1, &hi1, &lo2, &hi2);
            if (i1 < lo1 || i1 > hi1 || i2 < lo2 || i2 > hi2) continue;
            acc += beam_term(coef + 2 * b, y, eps, o1 + i1 * d1, o2 + i2 * d2);
        }
        out_re[k] = creal(acc);
        if (out_im) out_im[k] = cimag(acc);
    }
}

int or_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
