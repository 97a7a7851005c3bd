// Step 2 of the FGA algorithm on gfx950: classical RK4 of the ray equations
// (characline eq.) for H = sigma c(Q)|P| (hamiltonian eq.), of the dynamic
// ray tracing equations for A = dzQ, B = dzP (dzQ, dzP eqs.), of the action
// S and of the amplitude a (a_formu eq.).
//
// One thread owns one beam for all steps: the 23-double state and the RK4
// accumulators stay in VGPRs, so HBM sees one read and one write of the
// state per launch.  c and its derivatives come from the cubic B-spline of
// the velocity samples, evaluated as the bicubic polynomial of the knot cell
// (16 coefficients per cell, formed once per velocity model).  The
// coefficients of the next evaluation are requested as soon as its position
// is known (right after the slope of Q), straight into LDS with
// global_load_lds, so the cache latency overlaps the rest of the stage
// without holding VGPRs.
// FP64 throughout: gfx950 runs FP64 FMA at the FP32 rate, and the phase
// P.(x-Q)/eps needs Q and P to ~1e-14.
#include <limits.h>

#include "fga_internal.h"

#include "rk4.h"

#define RK_BLOCK 256

typedef __attribute__((address_space(3))) void lds_void;

// The eight transfers of one request for the lanes in mask: the 128 bytes at
// a, 16 per transfer, into the slots at LDS address lds, 1 KB apart.  A
// transfer lands at M0 + instruction offset + 16 lane and reads address +
// instruction offset, so one address register serves all eight: transfer s
// takes offset 16 s and M0 = lds + 1024 s - 16 s.  Written as one block so
// that the EXEC change leaves no branch in the compiled loop (a branch there
// makes the register allocator spill the RK4 state); each M0 write is
// followed by the wait state that an LDS transfer after it requires.  No
// VGPR receives data.
__device__ __forceinline__ void cell_dma(const double *a, unsigned lds, unsigned long long mask)
{
    unsigned long long saved;
    asm volatile(
        "s_and_saveexec_b64 %0, %2\n\t"
        "s_mov_b32 m0, %3\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off\n\t"
        "s_add_u32 m0, %3, 0x3f0\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:16\n\t"
        "s_add_u32 m0, %3, 0x7e0\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:32\n\t"
        "s_add_u32 m0, %3, 0xbd0\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:48\n\t"
        "s_add_u32 m0, %3, 0xfc0\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:64\n\t"
        "s_add_u32 m0, %3, 0x13b0\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:80\n\t"
        "s_add_u32 m0, %3, 0x17a0\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:96\n\t"
        "s_add_u32 m0, %3, 0x1b90\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %1, off offset:112\n\t"
        "s_mov_b64 exec, %0"
        : "=&s"(saved)
        : "v"(a), "s"(mask), "s"(lds)
        : "m0", "scc", "memory");
}

// Velocity source of the RK4 stages: prefetch() sends the 16 polynomial
// coefficients of the knot cell of (x1, x2) (one 128-byte line) to this
// wavefront's LDS slots, as eight 16-byte transfers per lane; eval() waits
// for them and evaluates the bicubic.  Slot s holds coefficients 2s, 2s + 1,
// lane l at entry l.  A beam moves a fraction of a cell per stage, so a lane
// whose cell is the one its slots already hold requests nothing, and the
// cache -> CU traffic, which bounds this loop otherwise, drops several-fold.
// (The table is 16 times the velocity grid and does not stay in the L2, but
// at this request rate one line per request and the shorter evaluation win
// over the 16 taps of the padded grid.)  The wavefront issues no other
// vector-memory load inside the step loop, so waiting for every outstanding
// one waits exactly for these.  Every evaluation is at the position of the
// request before it, so the cell and offsets found by prefetch() are kept
// and eval() does not locate the cell again (its position arguments are
// that same point).
struct VelDma {
    VelGrid V;
    double2 *buf;   // this wavefront's 8 slots of 64 entries
    int lane;
    int cur1, cur2;   // knot cell whose coefficients the slots hold (none at first)
    double f1, f2;    // offsets in that cell of the requested position
    __device__ __forceinline__ void prefetch(double x1, double x2)
    {
        const VelCell k = vel_cell(V, x1, x2);
        const bool changed = k.i1 != cur1 || k.i2 != cur2;
        cur1 = k.i1;
        cur2 = k.i2;
        f1 = k.f1;
        f2 = k.f2;
        cell_dma(vel_cell_coef(V, k), (unsigned)(size_t)(lds_void *)buf, __ballot(changed));
    }
    __device__ __forceinline__ void eval(double, double, double &c, double &c1, double &c2,
                                         double &c11, double &c12, double &c22) const
    {
        // the LDS writes of global_load_lds complete with the load counter
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const VelCell k = {cur1, cur2, f1, f2};
        double C[4][4];
#pragma unroll
        for (int sl = 0; sl < 8; ++sl) {
            const double2 v = buf[sl * 64 + lane];
            C[sl >> 1][2 * (sl & 1)] = v.x;
            C[sl >> 1][2 * (sl & 1) + 1] = v.y;
        }
        vel_poly(V, k, C, c, c1, c2, c11, c12, c22);
    }
};

// Principal square root of x + iy (|z| > 0), in the cancellation-free form.
__device__ __forceinline__ Cd csqrt_principal(Cd z)
{
    const double m = sqrt(fma(z.r, z.r, z.i * z.i));
    const double t = sqrt(0.5 * (fabs(z.r) + m));
    const double h = 0.5 * z.i / t;
    return z.r >= 0.0 ? Cd{t, h} : Cd{fabs(h), copysign(t, z.i)};
}

// (det Z)^{1/2} of the state, Z = A + iB, the root taken nearest prev.
__device__ __forceinline__ Cd det_root(const St &y, Cd prev)
{
    Cd Z[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l)
            Z[j][l] = {y.A[j][l].r - y.B[j][l].i, y.A[j][l].i + y.B[j][l].r};
    const Cd r = csqrt_principal(csub(cmul(Z[0][0], Z[1][1]), cmul(Z[0][1], Z[1][0])));
    return r.r * prev.r + r.i * prev.i < 0.0 ? Cd{-r.r, -r.i} : r;
}

// One thread per beam; the state, the RK4 accumulator and the stage input
// live in VGPRs (two wavefronts per SIMD), the cell coefficients in 8 KB of
// LDS per wavefront.  CLOSED: the amplitude is not integrated; the root of
// det Z is followed step by step (recovered at the start from the incoming
// a = c(Q)/c(q) root, 2 at t = 0), and a = c(Q)/c(q) root at the end.
// ckpt (if not null) receives the incoming state, or with EVERY the state
// before every step and the final one, ckpt[nsteps + 1][NSTATE][cap].
template <bool CLOSED, bool EVERY = false>
__global__ void __launch_bounds__(RK_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_rk4(VelGrid V, double *__restrict__ f, const int64_t *__restrict__ id,
      const int64_t *__restrict__ offsets, int nshots, int64_t cap, int64_t NqNp, double dt,
      int nsteps, double *__restrict__ ckpt, int64_t *status)
{
    __shared__ double2 slots[RK_BLOCK / 64][8 * 64];
    const int tid = threadIdx.x;
    // the wavefront index is uniform: keep the LDS base in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    VelDma vel{V, slots[wave], tid & 63, INT_MIN, INT_MIN, 0.0, 0.0};
    int64_t nb = offsets[nshots];
    for (int64_t b0 = (int64_t)blockIdx.x * RK_BLOCK; b0 < nb;
         b0 += (int64_t)gridDim.x * RK_BLOCK) {
        int64_t b = b0 + tid;
        if (b >= nb) continue;
        St y;
        load_state(f, cap, b, y);
        if (ckpt && !EVERY) store_state(ckpt + b, cap, y);
        // H of branch - is -H of branch +, so every slope of the - branch is
        // exactly the negative of the + branch's: the stages run the + branch
        // with signed steps (bit-identical to signed slopes, no sign products)
        const double s = ((id[b] / NqNp) & 1) ? -1.0 : 1.0;
        const double sdt = s * dt;
        const double h2 = 0.5 * sdt, h6 = sdt / 6.0, h3 = sdt / 3.0;
        double cq = 1.0;
        Cd root = {0.0, 0.0};
        if (CLOSED) {
            double c0, d[5];
            vel_eval(V, f[b], f[cap + b], cq, d[0], d[1], d[2], d[3], d[4]);
            vel_eval(V, y.Q1, y.Q2, c0, d[0], d[1], d[2], d[3], d[4]);
            root = cscale(y.a, cq / c0);
        }
        vel.cur1 = vel.cur2 = INT_MIN;   // new beam: its slots hold nothing yet
        if (nsteps > 0) vel.prefetch(y.Q1, y.Q2);
        for (int it = 0; it < nsteps; ++it) {
            if (EVERY) store_state(ckpt + (size_t)it * FGA_NSTATE * cap + b, cap, y);
            St t = y, acc = y;
            rk_stage<false, VelDma, !CLOSED>(vel, 1.0, t, acc, y, h6, h2);
            rk_stage<false, VelDma, !CLOSED>(vel, 1.0, t, acc, y, h3, h2);
            rk_stage<false, VelDma, !CLOSED>(vel, 1.0, t, acc, y, h3, sdt);
            rk_stage<true, VelDma, !CLOSED>(vel, 1.0, t, acc, y, h6, 0.0);
            y = acc;
            if (CLOSED) root = det_root(y, root);
        }
        if (EVERY) store_state(ckpt + (size_t)nsteps * FGA_NSTATE * cap + b, cap, y);
        if (CLOSED && nsteps > 0) {
            // the last stage requested the coefficients at the final position
            double cQ, d[5];
            vel.eval(y.Q1, y.Q2, cQ, d[0], d[1], d[2], d[3], d[4]);
            y.a = cscale(root, cQ / cq);
        }
        // no LDS transfer (the last step requests one more) may outlive the
        // wavefront's use of the slots
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (!isfinite(y.Q1) || !isfinite(y.Q2) || !isfinite(y.a.r) || !isfinite(y.a.i))
            atomicOr((unsigned long long *)status, FGA_STATUS_NUMERIC);
        store_state(f + (size_t)FGA_F_STATE * cap + b, cap, y);
    }
}

// ---------------------------------------------------------------------------
// Divided-difference mode: dzQ and dzP from the rays of the neighbouring mesh
// nodes instead of the dynamic ray tracing equations.
//
// One lane per ray: lanes 9m .. 9m + 8 of a wavefront carry beam m of the
// wavefront's seven (role 0: the beam's own ray; roles 1 + 2r and 2 + 2r:
// the rays displaced by +h_r and -h_r along direction r = q1, q2, p1, p2;
// lane 63 repeats lane 54's ray and stores nothing).  A lane holds only the
// five ray values, so the state of the RK4 is small; the cell coefficients
// come through the same LDS prefetch as in k_rk4.  After every step the
// lanes put Q and P into LDS and every lane reads the eight neighbours of its
// beam, forms Z = dzQ + i dzP from the central differences and follows the
// root of det Z; the beam's own lane finally stores Q, P, S, A, B and
// a = c(Q)/c(q) root.

#define DD_BEAMS 7   // beams per wavefront (9 lanes each)

struct Ray {
    double Q1, Q2, P1, P2, S;
};

// One RK4 stage of the characteristic equations and the action alone,
// fused like rk_stage: k = f(t), acc += wacc k, t = y + hnext k.
template <bool LAST, class Vel>
__device__ __forceinline__ void ray_stage(Vel &vel, double s, Ray &t, Ray &acc, const Ray &y,
                                          double wacc, double hnext)
{
    double c, g1, g2, K11, K12, K22;
    vel.eval(t.Q1, t.Q2, c, g1, g2, K11, K12, K22);
    const double n2 = fma(t.P1, t.P1, t.P2 * t.P2);
    const double inv_n = rsq64(n2);
    const double n = n2 * inv_n;
    const double sc = s * c;
    const double kQ1 = sc * (t.P1 * inv_n), kQ2 = sc * (t.P2 * inv_n);
    const double kP1 = -s * n * g1, kP2 = -s * n * g2;
    const double kS = t.P1 * kQ1 + t.P2 * kQ2 - sc * n;
    acc.Q1 = fma(wacc, kQ1, acc.Q1);
    acc.Q2 = fma(wacc, kQ2, acc.Q2);
    acc.P1 = fma(wacc, kP1, acc.P1);
    acc.P2 = fma(wacc, kP2, acc.P2);
    acc.S = fma(wacc, kS, acc.S);
    if (LAST) {
        vel.prefetch(acc.Q1, acc.Q2);
    } else {
        t.Q1 = fma(hnext, kQ1, y.Q1);
        t.Q2 = fma(hnext, kQ2, y.Q2);
        vel.prefetch(t.Q1, t.Q2);
        t.P1 = fma(hnext, kP1, y.P1);
        t.P2 = fma(hnext, kP2, y.P2);
        t.S = fma(hnext, kS, y.S);
    }
}

// dzQ, dzP of the beam whose lanes start at lane `first`, from the rays in
// LDS (xq: Q, xp: P of each lane): dq_j = (+q_j - -q_j) inv2h[j],
// dp_j = (+p_j - -p_j) inv2h[2 + j]; A[j][k] = dq_j Q_k - i dp_j Q_k,
// B[j][k] = dq_j P_k - i dp_j P_k.
__device__ __forceinline__ void dd_AB(const double2 *xq, const double2 *xp, int first,
                                      const double inv2h[4], Cd A[2][2], Cd B[2][2])
{
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double2 qa = xq[first + 1 + 2 * j], qb = xq[first + 2 + 2 * j];
        const double2 qc = xq[first + 5 + 2 * j], qd = xq[first + 6 + 2 * j];
        const double2 pa = xp[first + 1 + 2 * j], pb = xp[first + 2 + 2 * j];
        const double2 pc = xp[first + 5 + 2 * j], pd = xp[first + 6 + 2 * j];
        const double hq = inv2h[j], hp = inv2h[2 + j];
        A[j][0] = {(qa.x - qb.x) * hq, -(qc.x - qd.x) * hp};
        A[j][1] = {(qa.y - qb.y) * hq, -(qc.y - qd.y) * hp};
        B[j][0] = {(pa.x - pb.x) * hq, -(pc.x - pd.x) * hp};
        B[j][1] = {(pa.y - pb.y) * hq, -(pc.y - pd.y) * hp};
    }
}

__device__ __forceinline__ Cd det_Z(const Cd A[2][2], const Cd B[2][2])
{
    Cd Z[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int l = 0; l < 2; ++l) Z[j][l] = {A[j][l].r - B[j][l].i, A[j][l].i + B[j][l].r};
    return csub(cmul(Z[0][0], Z[1][1]), cmul(Z[0][1], Z[1][0]));
}

__global__ void __launch_bounds__(RK_BLOCK)
k_rk4_dd(VelGrid V, double *__restrict__ f, const int64_t *__restrict__ id,
         const int64_t *__restrict__ offsets, int nshots, int64_t cap, int64_t NqNp, double dt,
         int nsteps, double4 hmesh, double *__restrict__ ckpt, int64_t *status)
{
    __shared__ double2 slots[RK_BLOCK / 64][8 * 64];
    __shared__ double2 xq[RK_BLOCK / 64][64], xp[RK_BLOCK / 64][64];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int m = lane == 63 ? DD_BEAMS - 1 : lane / 9;       // beam of the lane in the wave
    const int role = lane == 63 ? 0 : lane % 9;
    const int first = 9 * m;
    const bool owner = role == 0 && lane != 63;
    const double h[4] = {hmesh.x, hmesh.y, hmesh.z, hmesh.w};
    const double inv2h[4] = {0.5 / hmesh.x, 0.5 / hmesh.y, 0.5 / hmesh.z, 0.5 / hmesh.w};
    // displacement of this lane's ray: direction r, side +-1 (none for role 0)
    const int r = role == 0 ? 0 : (role - 1) >> 1;
    const double hs = role == 0 ? 0.0 : (((role - 1) & 1) ? -h[r] : h[r]);
    const int dj = r & 1;
    const bool alongp = r >= 2;
    VelDma vel{V, slots[wave], lane, INT_MIN, INT_MIN, 0.0, 0.0};
    double2 *wq = xq[wave], *wp = xp[wave];
    const int64_t nb = offsets[nshots];
    const int64_t per_block = (int64_t)(RK_BLOCK / 64) * DD_BEAMS;
    for (int64_t b0 = (int64_t)blockIdx.x * per_block; b0 < nb;
         b0 += (int64_t)gridDim.x * per_block) {
        const int64_t wb = b0 + (int64_t)wave * DD_BEAMS;
        if (wb >= nb) continue;                                 // uniform in the wavefront
        const int64_t braw = wb + m;
        const bool valid = braw < nb;
        const int64_t b = valid ? braw : nb - 1;
        const double *st = f + (size_t)FGA_F_STATE * cap + b;
        if (ckpt && owner && valid)
            for (int k = 0; k < FGA_NSTATE; ++k) ckpt[(size_t)k * cap + b] = st[(size_t)k * cap];
        // the displaced ray starts along the incoming A, B:
        // dq_j Q_k = Re A[j][k], dp_j Q_k = -Im A[j][k] (P alike with B)
        const int fa = 5 + 4 * dj + (alongp ? 1 : 0);
        const double sg = alongp ? -hs : hs;
        Ray y;
        y.Q1 = fma(sg, st[(size_t)fa * cap], st[0]);
        y.Q2 = fma(sg, st[(size_t)(fa + 2) * cap], st[cap]);
        y.P1 = fma(sg, st[(size_t)(fa + 8) * cap], st[2 * cap]);
        y.P2 = fma(sg, st[(size_t)(fa + 10) * cap], st[3 * cap]);
        y.S = st[4 * cap];
        // branch - runs as branch + with signed steps (as in k_rk4)
        const double sdt = ((id[b] / NqNp) & 1) ? -dt : dt;
        const double h2 = 0.5 * sdt, h6 = sdt / 6.0, h3 = sdt / 3.0;
        double cq, c0, d[5];
        vel_eval(V, f[b], f[cap + b], cq, d[0], d[1], d[2], d[3], d[4]);
        vel_eval(V, st[0], st[cap], c0, d[0], d[1], d[2], d[3], d[4]);
        Cd root = cscale(Cd{st[21 * cap], st[22 * cap]}, cq / c0);
        vel.cur1 = vel.cur2 = INT_MIN;
        vel.prefetch(y.Q1, y.Q2);
        for (int it = 0; it < nsteps; ++it) {
            Ray t = y, acc = y;
            ray_stage<false>(vel, 1.0, t, acc, y, h6, h2);
            ray_stage<false>(vel, 1.0, t, acc, y, h3, h2);
            ray_stage<false>(vel, 1.0, t, acc, y, h3, sdt);
            ray_stage<true>(vel, 1.0, t, acc, y, h6, 0.0);
            y = acc;
            // exchange within the wavefront: the previous step's reads are
            // done before these writes, and these writes before the reads
            __builtin_amdgcn_wave_barrier();
            wq[lane] = double2{y.Q1, y.Q2};
            wp[lane] = double2{y.P1, y.P2};
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            Cd A[2][2], B[2][2];
            dd_AB(wq, wp, first, inv2h, A, B);
            const Cd rt = csqrt_principal(det_Z(A, B));
            root = rt.r * root.r + rt.i * root.i < 0.0 ? Cd{-rt.r, -rt.i} : rt;
        }
        double cQ;
        vel.eval(y.Q1, y.Q2, cQ, d[0], d[1], d[2], d[3], d[4]);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (owner && valid) {
            St o;
            o.Q1 = y.Q1;
            o.Q2 = y.Q2;
            o.P1 = y.P1;
            o.P2 = y.P2;
            o.S = y.S;
            dd_AB(wq, wp, first, inv2h, o.A, o.B);
            o.a = cscale(root, cQ / cq);
            if (!isfinite(o.Q1) || !isfinite(o.Q2) || !isfinite(o.a.r) || !isfinite(o.a.i))
                atomicOr((unsigned long long *)status, FGA_STATUS_NUMERIC);
            store_state(f + (size_t)FGA_F_STATE * cap + b, cap, o);
        }
        // the next beam's first exchange must not overwrite what is read here
        __builtin_amdgcn_wave_barrier();
    }
}

fga_status fga_launch_propagate(fga_ctx *ctx, fga_beams *beams, int nshots, int nsteps,
                                double *ckpt)
{
    VelGrid V = fga_velgrid(ctx);
    int64_t NqNp = (int64_t)ctx->p.nq1 * ctx->p.nq2 * ctx->p.np1 * ctx->p.np2;
    // persistent grid: the beam count lives on the device
    int blocks = ctx->num_cu * 8;
    if (ctx->p.dz_divided) {
        if (nsteps <= 0) return FGA_OK;
        const fga_grid &g = ctx->g;
        const double sc = ctx->p.dz_scale;
        double4 hm = make_double4(sc * (ctx->p.qs1 * g.d1), sc * (ctx->p.qs2 * g.d2),
                                  sc * ctx->p.dp1, sc * ctx->p.dp2);
        hipLaunchKernelGGL(k_rk4_dd, dim3(blocks), dim3(RK_BLOCK), 0, ctx->stream, V, beams->f,
                           beams->id, beams->offsets, nshots, beams->capacity, NqNp, ctx->p.dt,
                           nsteps, hm, ckpt, ctx->status);
    } else if (ctx->p.amp_closed)
        hipLaunchKernelGGL(k_rk4<true>, dim3(blocks), dim3(256), 0, ctx->stream, V, beams->f,
                           beams->id, beams->offsets, nshots, beams->capacity, NqNp, ctx->p.dt,
                           nsteps, ckpt, ctx->status);
    else if (ckpt && ctx->p.ckpt_every_step)
        hipLaunchKernelGGL((k_rk4<false, true>), dim3(blocks), dim3(256), 0, ctx->stream, V,
                           beams->f, beams->id, beams->offsets, nshots, beams->capacity, NqNp,
                           ctx->p.dt, nsteps, ckpt, ctx->status);
    else
        hipLaunchKernelGGL(k_rk4<false>, dim3(blocks), dim3(256), 0, ctx->stream, V, beams->f,
                           beams->id, beams->offsets, nshots, beams->capacity, NqNp, ctx->p.dt,
                           nsteps, ckpt, ctx->status);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}
