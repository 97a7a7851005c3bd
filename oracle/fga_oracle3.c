/* Plain FP64 CPU oracle of the frozen Gaussian approximation in three space
 * dimensions (test infrastructure: only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call it; it shares no code with the HIP
 * path).  The paper states the method for general d; here d = 3:
 *   - the velocity: tricubic B-spline with the samples as coefficients,
 *     indices clamped to the grid;
 *   - step 1: psi(q,p) of the psi eq. as a Riemann sum over the box B_eps;
 *   - step 2: classical RK4 of the characteristic equations for
 *     H = sigma c(Q)|P|, the dynamic ray tracing equations for the 3x3
 *     complex matrices A = dzQ, B = dzP and the amplitude equation
 *     (a_formu eq.), Z^{-1} by the 3x3 adjugate;
 *   - step 3: the recons eq. over the truncation box of every beam.
 * State layout (45 doubles): Q1 Q2 Q3 | P1 P2 P3 | S | A[j][k] (re, im),
 * row-major | B[j][k] (re, im) | a (re, im). */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define NST3 45

/* cubic B-spline beta3(s) and its first two derivatives */
static double b3(double s, int deriv)
{
    double a = fabs(s), sg = (s < 0.0) ? -1.0 : 1.0;
    if (a < 1.0) {
        if (deriv == 0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (deriv == 1) return sg * (-2.0 * a + 1.5 * a * a);
        return -2.0 + 3.0 * a;
    }
    if (a < 2.0) {
        double b = 2.0 - a;
        if (deriv == 0) return b * b * b / 6.0;
        if (deriv == 1) return -sg * 0.5 * b * b;
        return b;
    }
    return 0.0;
}

static int clamp3(int k, int n) { return k < 0 ? 0 : (k > n - 1 ? n - 1 : k); }

typedef struct {
    const double *c;
    int n[3];
    double o[3], d[3];
} vel3_t;

/* out = {c, c_1, c_2, c_3, c_11, c_12, c_13, c_22, c_23, c_33} at x:
 * sum over the 4 x 4 x 4 knots around x of c_k times the product of the
 * three beta3 factors (differentiated as the output entry asks). */
static void vel3(const vel3_t *v, const double *x, double *out)
{
    static const int D[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                 {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
    double w[3][3][4];
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        double t = (x[a] - v->o[a]) / v->d[a];
        i0[a] = (int)floor(t);
        for (int dd = 0; dd < 3; ++dd)
            for (int k = 0; k < 4; ++k)
                w[a][dd][k] = b3(t - (i0[a] - 1 + k), dd) / pow(v->d[a], dd);
    }
    for (int r = 0; r < 10; ++r) out[r] = 0.0;
    for (int k3 = 0; k3 < 4; ++k3)
        for (int k2 = 0; k2 < 4; ++k2)
            for (int k1 = 0; k1 < 4; ++k1) {
                double ck = v->c[((size_t)clamp3(i0[2] - 1 + k3, v->n[2]) * v->n[1] +
                                  clamp3(i0[1] - 1 + k2, v->n[1])) * v->n[0] +
                                 clamp3(i0[0] - 1 + k1, v->n[0])];
                for (int r = 0; r < 10; ++r)
                    out[r] += ck * w[0][D[r][0]][k1] * w[1][D[r][1]][k2] * w[2][D[r][2]][k3];
            }
}

void or3_velocity_points(const double *c, int n1, int n2, int n3, double o1, double o2,
                         double o3, double d1, double d2, double d3, int64_t npts,
                         const double *x, double *out)
{
    vel3_t v = {c, {n1, n2, n3}, {o1, o2, o3}, {d1, d2, d3}};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) vel3(&v, x + 3 * i, out + 10 * i);
}

static int halfwidth3(double eps, double tau, double d)
{
    return (int)ceil(sqrt(2.0 * eps * log(1.0 / tau)) / d);
}

static double pnode(int l, int np, double dp) { return (l - 0.5 * (np - 1)) * dp; }

/* psi(q,p) = d1 d2 d3 sum_m f(k+m) exp(-|m d|^2/(2 eps) - i p.(m d)/eps) over
 * the box, for q = (qb_a + j_a qs_a) and the staggered p-mesh.
 * psi[((jq * Np) + lp) * 2 + {re, im}], jq = (j3 nq2 + j2) nq1 + j1,
 * lp = (l3 np2 + l2) np1 + l1.  f: [n3][n2][n1]. */
void or3_fbi(const double *f, const int *n, const double *d, double eps, double tau_fbi,
             const int *qb, const int *qs, const int *nq, const int *np, const double *dp,
             double *psi)
{
    int R[3], W[3];
    double complex *E[3];
    for (int a = 0; a < 3; ++a) {
        R[a] = halfwidth3(eps, tau_fbi, d[a]);
        W[a] = 2 * R[a] + 1;
        E[a] = malloc(sizeof(double complex) * (size_t)np[a] * W[a]);
        for (int l = 0; l < np[a]; ++l)
            for (int m = -R[a]; m <= R[a]; ++m) {
                double r = m * d[a];
                E[a][(size_t)l * W[a] + m + R[a]] =
                    exp(-r * r / (2.0 * eps)) * cexp(-I * pnode(l, np[a], dp[a]) * r / eps);
            }
    }
    const int64_t NQ = (int64_t)nq[0] * nq[1] * nq[2], NP = (int64_t)np[0] * np[1] * np[2];
#pragma omp parallel for collapse(2) schedule(dynamic, 8)
    for (int64_t jq = 0; jq < NQ; ++jq)
        for (int64_t lp = 0; lp < NP; ++lp) {
            int j1 = (int)(jq % nq[0]), j2 = (int)((jq / nq[0]) % nq[1]),
                j3 = (int)(jq / ((int64_t)nq[0] * nq[1]));
            int l1 = (int)(lp % np[0]), l2 = (int)((lp / np[0]) % np[1]),
                l3 = (int)(lp / ((int64_t)np[0] * np[1]));
            int k1 = qb[0] + j1 * qs[0], k2 = qb[1] + j2 * qs[1], k3 = qb[2] + j3 * qs[2];
            const double complex *e1 = E[0] + (size_t)l1 * W[0];
            const double complex *e2 = E[1] + (size_t)l2 * W[1];
            const double complex *e3 = E[2] + (size_t)l3 * W[2];
            double complex acc = 0.0;
            for (int m3 = -R[2]; m3 <= R[2]; ++m3) {
                int y3 = k3 + m3;
                if (y3 < 0 || y3 >= n[2]) continue;
                double complex a2 = 0.0;
                for (int m2 = -R[1]; m2 <= R[1]; ++m2) {
                    int y2 = k2 + m2;
                    if (y2 < 0 || y2 >= n[1]) continue;
                    const double *row = f + ((size_t)y3 * n[1] + y2) * n[0];
                    double complex a1 = 0.0;
                    for (int m1 = -R[0]; m1 <= R[0]; ++m1) {
                        int y1 = k1 + m1;
                        if (y1 < 0 || y1 >= n[0]) continue;
                        a1 += row[y1] * e1[m1 + R[0]];
                    }
                    a2 += e2[m2 + R[1]] * a1;
                }
                acc += e3[m3 + R[2]] * a2;
            }
            acc *= d[0] * d[1] * d[2];
            psi[(jq * NP + lp) * 2 + 0] = creal(acc);
            psi[(jq * NP + lp) * 2 + 1] = cimag(acc);
        }
    for (int a = 0; a < 3; ++a) free(E[a]);
}

/* Right-hand side of the characteristic, dynamic ray tracing, action and
 * amplitude equations for H = sigma c(Q)|P| in three dimensions:
 *   dQ = H_P, dP = -H_Q, dS = P.H_P - H,
 *   dA = A H_QP + B H_PP, dB = -A H_QQ - B H_PQ  ((j,k) entry d/dz_j of Q_k),
 *   da = a [ (H_P.H_Q)/H + tr(Z^{-1} dZ)/2 ],  Z = A + iB. */
static void rhs3(const vel3_t *v, double sigma, const double *y, double *dy)
{
    double cv[10];
    vel3(v, y, cv);
    double c = cv[0], g[3] = {cv[1], cv[2], cv[3]};
    double K[3][3] = {{cv[4], cv[5], cv[6]}, {cv[5], cv[7], cv[8]}, {cv[6], cv[8], cv[9]}};
    const double *P = y + 3;
    double n = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
    double u[3] = {P[0] / n, P[1] / n, P[2] / n};
    double H = sigma * c * n;
    double HP[3], HQ[3], HPP[3][3], HQQ[3][3], HQP[3][3], HPQ[3][3];
    for (int l = 0; l < 3; ++l) {
        HP[l] = sigma * c * u[l];
        HQ[l] = sigma * n * g[l];
        for (int k = 0; k < 3; ++k) {
            HPP[l][k] = sigma * (c / n) * ((l == k ? 1.0 : 0.0) - u[l] * u[k]);
            HQQ[l][k] = sigma * n * K[l][k];
            HQP[l][k] = sigma * g[l] * u[k];
            HPQ[l][k] = sigma * u[l] * g[k];
        }
    }
    for (int l = 0; l < 3; ++l) {
        dy[l] = HP[l];
        dy[3 + l] = -HQ[l];
    }
    dy[6] = P[0] * HP[0] + P[1] * HP[1] + P[2] * HP[2] - H;
    double complex A[3][3], B[3][3], dA[3][3], dB[3][3], Z[3][3], dZ[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            A[j][k] = y[7 + 2 * (3 * j + k)] + I * y[8 + 2 * (3 * j + k)];
            B[j][k] = y[25 + 2 * (3 * j + k)] + I * y[26 + 2 * (3 * j + k)];
        }
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            double complex sa = 0.0, sb = 0.0;
            for (int l = 0; l < 3; ++l) {
                sa += A[j][l] * HQP[l][k] + B[j][l] * HPP[l][k];
                sb += -A[j][l] * HQQ[l][k] - B[j][l] * HPQ[l][k];
            }
            dA[j][k] = sa;
            dB[j][k] = sb;
            dy[7 + 2 * (3 * j + k)] = creal(sa);
            dy[8 + 2 * (3 * j + k)] = cimag(sa);
            dy[25 + 2 * (3 * j + k)] = creal(sb);
            dy[26 + 2 * (3 * j + k)] = cimag(sb);
            Z[j][k] = A[j][k] + I * B[j][k];
            dZ[j][k] = sa + I * sb;
        }
    /* Z^{-1} = adj(Z) / det Z; adj(Z)[k][j] is the (j,k) cofactor */
    double complex cof[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            int j1 = (j + 1) % 3, j2 = (j + 2) % 3, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            cof[j][k] = Z[j1][k1] * Z[j2][k2] - Z[j1][k2] * Z[j2][k1];
        }
    double complex det = Z[0][0] * cof[0][0] + Z[0][1] * cof[0][1] + Z[0][2] * cof[0][2];
    double complex tr = 0.0;
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) tr += cof[j][k] * dZ[j][k];   /* (adj Z)[k][j] dZ[j][k] */
    tr /= det;
    double complex a = y[43] + I * y[44];
    double complex da = a * (HP[0] * HQ[0] + HP[1] * HQ[1] + HP[2] * HQ[2]) / H + 0.5 * a * tr;
    dy[43] = creal(da);
    dy[44] = cimag(da);
}

void or3_rhs(const double *c, const int *n, const double *o, const double *d, double sigma,
             const double *y, double *dy)
{
    vel3_t v = {c, {n[0], n[1], n[2]}, {o[0], o[1], o[2]}, {d[0], d[1], d[2]}};
    rhs3(&v, sigma, y, dy);
}

/* classical RK4, fixed dt, nsteps steps, every beam independently */
void or3_propagate(const double *c, const int *n, const double *o, const double *d, int64_t nb,
                   const int8_t *sigma, double *state, double dt, int nsteps)
{
    vel3_t v = {c, {n[0], n[1], n[2]}, {o[0], o[1], o[2]}, {d[0], d[1], d[2]}};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
        double *y = state + (size_t)b * NST3;
        double s = (double)sigma[b];
        double k1[NST3], k2[NST3], k3[NST3], k4[NST3], t[NST3];
        for (int it = 0; it < nsteps; ++it) {
            rhs3(&v, s, y, k1);
            for (int i = 0; i < NST3; ++i) t[i] = y[i] + 0.5 * dt * k1[i];
            rhs3(&v, s, t, k2);
            for (int i = 0; i < NST3; ++i) t[i] = y[i] + 0.5 * dt * k2[i];
            rhs3(&v, s, t, k3);
            for (int i = 0; i < NST3; ++i) t[i] = y[i] + dt * k3[i];
            rhs3(&v, s, t, k4);
            for (int i = 0; i < NST3; ++i)
                y[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        }
    }
}

/* u(x) = Re sum_b C_b a_b exp(i S_b/eps) exp(i P_b.(x - Q_b)/eps - |x - Q_b|^2/(2 eps))
 * over the beams whose box (half-width Rw_a around the node nearest Q)
 * holds x.  coef: [nb][2]; state: [nb][45]; u: [n3][n2][n1], overwritten. */
void or3_reconstruct(const int *n, const double *o, const double *d, double eps,
                     double tau_win, int64_t nb, const double *coef, const double *state,
                     double *u)
{
    int Rw[3];
    for (int a = 0; a < 3; ++a) Rw[a] = halfwidth3(eps, tau_win, d[a]);
    const int64_t N = (int64_t)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) u[i] = 0.0;
    /* beams in order, each writing only its box: a node's sum runs over the
     * beams in beam order */
    for (int64_t b = 0; b < nb; ++b) {
        const double *y = state + (size_t)b * NST3;
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            double t = floor((y[a] - o[a]) / d[a] + 0.5);
            t = fmin(fmax(t, -1e8), 1e8);
            int cn = (int)t;
            lo[a] = cn - Rw[a] < 0 ? 0 : cn - Rw[a];
            hi[a] = cn + Rw[a] > n[a] - 1 ? n[a] - 1 : cn + Rw[a];
        }
        double complex Ca = (coef[2 * b] + I * coef[2 * b + 1]) * (y[43] + I * y[44]);
#pragma omp parallel for collapse(2) schedule(static)
        for (int i3 = lo[2]; i3 <= hi[2]; ++i3)
            for (int i2 = lo[1]; i2 <= hi[1]; ++i2)
                for (int i1 = lo[0]; i1 <= hi[0]; ++i1) {
                    double r[3] = {o[0] + i1 * d[0] - y[0], o[1] + i2 * d[1] - y[1],
                                   o[2] + i3 * d[2] - y[2]};
                    double ph = (y[6] + y[3] * r[0] + y[4] * r[1] + y[5] * r[2]) / eps;
                    double ga = -(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) / (2.0 * eps);
                    u[((size_t)i3 * n[1] + i2) * n[0] + i1] += creal(Ca * cexp(I * ph + ga));
                }
    }
}
