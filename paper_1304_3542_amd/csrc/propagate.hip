// Step 2 of the FGA algorithm on gfx950: classical RK4 of the ray equations
// (characline eq.) for H = sigma c(Q)|P| (hamiltonian eq.), of the dynamic
// ray tracing equations for A = dzQ, B = dzP (dzQ, dzP eqs.), of the action
// S and of the amplitude a (a_formu eq.).
//
// One thread owns one beam for all steps: the 23-double state and the RK4
// accumulators stay in VGPRs, so HBM sees one read and one write of the
// state per launch.  c and its derivatives come from the cubic B-spline of
// the velocity samples (16 taps per evaluation), read through the L2 (the
// velocity grid is a few MB and stays cache resident).  FP64 throughout:
// gfx950 runs FP64 FMA at the FP32 rate, and the phase P.(x-Q)/eps needs Q
// and P to ~1e-14.
#include "fga_internal.h"

#include "rk4.h"

#define RK_BLOCK 256

// One thread per beam; the state, the RK4 accumulator and the stage input
// live in VGPRs (two wavefronts per SIMD).
__global__ void __launch_bounds__(RK_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_rk4(VelGrid V, double *__restrict__ f, const int64_t *__restrict__ id,
      const int64_t *__restrict__ offsets, int nshots, int64_t cap, int64_t NqNp, double dt,
      int nsteps, double *__restrict__ ckpt, int64_t *status)
{
    const int tid = threadIdx.x;
    int64_t nb = offsets[nshots];
    for (int64_t b0 = (int64_t)blockIdx.x * RK_BLOCK; b0 < nb;
         b0 += (int64_t)gridDim.x * RK_BLOCK) {
        int64_t b = b0 + tid;
        if (b >= nb) continue;
        St y;
        load_state(f, cap, b, y);
        if (ckpt) store_state(ckpt + b, cap, y);
        double s = ((id[b] / NqNp) & 1) ? -1.0 : 1.0;
        double h2 = 0.5 * dt, h6 = dt / 6.0, h3 = dt / 3.0;
        for (int it = 0; it < nsteps; ++it) {
            St t = y, acc = y;
            stage<false>(V, s, t, acc, y, h6, h2);
            stage<false>(V, s, t, acc, y, h3, h2);
            stage<false>(V, s, t, acc, y, h3, dt);
            stage<true>(V, s, t, acc, y, h6, 0.0);
            y = acc;
        }
        if (!isfinite(y.Q1) || !isfinite(y.Q2) || !isfinite(y.a.r) || !isfinite(y.a.i))
            atomicOr((unsigned long long *)status, FGA_STATUS_NUMERIC);
        store_state(f + (size_t)FGA_F_STATE * cap + b, cap, y);
    }
}

fga_status fga_launch_propagate(fga_ctx *ctx, fga_beams *beams, int nshots, int nsteps,
                                double *ckpt)
{
    VelGrid V = fga_velgrid(ctx);
    int64_t NqNp = (int64_t)ctx->p.nq1 * ctx->p.nq2 * ctx->p.np1 * ctx->p.np2;
    // persistent grid: the beam count lives on the device
    int blocks = ctx->num_cu * 8;
    hipLaunchKernelGGL(k_rk4, dim3(blocks), dim3(256), 0, ctx->stream, V, beams->f, beams->id,
                       beams->offsets, nshots, beams->capacity, NqNp, ctx->p.dt, nsteps, ckpt,
                       ctx->status);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}
