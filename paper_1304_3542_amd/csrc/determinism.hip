// Deterministic reduction of the dJ/dc logs of the adjoint kernels.
//
// In deterministic mode every beam writes the 16 knot sums of each knot cell
// it leaves (one record per flush) into its own log slots instead of adding
// them to dc with atomics.  The records are then summed in an order that does
// not depend on scheduling:
//   1. the log lengths are scanned into offsets (beam order),
//   2. the records are listed as (cell, log slot) in beam-then-sequence order
//      and sorted by cell with a stable radix sort, so every cell's records
//      stay in beam-then-sequence order,
//   3. one wavefront per cell sums its records (eight lanes per record, one
//      16-byte part each; lane group r takes every 8th record from the r-th,
//      in order; then a fixed butterfly over the groups),
//   4. one thread per grid knot adds the sums of the cells that reach it (the
//      clamped 4 x 4 knot stencil of the B-spline) in a fixed cell order.
// Integer atomics only count; every floating-point sum has a fixed order.
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "fga_internal.h"

// (nb, sum of log lengths, longest log) over the beams of the call
__global__ void k_det_stats(const int64_t *__restrict__ offsets, int nshots,
                            const int *__restrict__ cnt, unsigned long long *stats)
{
    const int64_t nb = offsets[nshots];
    unsigned long long tot = 0, mx = 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long c = (unsigned long long)cnt[b];
        tot += c;
        mx = c > mx ? c : mx;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) stats[0] = (unsigned long long)nb;
    if (tot) atomicAdd(&stats[1], tot);
    if (mx) atomicMax(&stats[2], mx);
}

__global__ void k_det_zero_u64(unsigned long long *p, int n)
{
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_det_zero_i32(int *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// (cell, slot) of every record, listed in beam order then log order.  A
// wavefront takes 64 consecutive beams, whose output ranges are consecutive.
// It reads a window of DL_K log positions of its beams into LDS (position k
// of consecutive beams is contiguous, so the reads are whole lines), then
// writes each beam's entries of the window to its range with consecutive
// lanes, so the stores are runs instead of one partial line per lane.
#define DL_K 32

__global__ void __launch_bounds__(256)
k_det_list(const int *__restrict__ cnt, const int64_t *__restrict__ off,
           const int *__restrict__ cell, int64_t nb, int64_t cap, unsigned *__restrict__ keys,
           unsigned long long *__restrict__ slots)
{
    __shared__ int win[4][DL_K][65];   // [wave][k][beam], padded against bank conflicts
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t b0 = ((int64_t)blockIdx.x * 4 + w) * 64; b0 < nb;
         b0 += (int64_t)gridDim.x * 256) {
        const int64_t b = b0 + lane;
        const int n = b < nb ? cnt[b] : 0;
        const int64_t o = b < nb ? off[b] : 0;
        int nmax = n;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) nmax = max(nmax, __shfl_xor(nmax, m, 64));
        for (int k0 = 0; k0 < nmax; k0 += DL_K) {
            const int kn = min(DL_K, nmax - k0);   // uniform
            for (int k = 0; k < kn; ++k)
                if (k0 + k < n) win[w][k][lane] = cell[(size_t)(k0 + k) * cap + b];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int j = 0; j < 64; ++j) {
                // beam j's count and offset (j is uniform: scalar reads of lane j)
                const int nj = __builtin_amdgcn_readlane(n, j);
                const int lo = __builtin_amdgcn_readlane((int)(unsigned)(o & 0xffffffff), j);
                const int hi = __builtin_amdgcn_readlane((int)(o >> 32), j);
                const int64_t oj = (int64_t)(((unsigned long long)(unsigned)hi << 32) |
                                             (unsigned long long)(unsigned)lo);
                if (lane < min(nj - k0, kn)) {
                    const int64_t q = oj + k0 + lane;
                    keys[q] = (unsigned)win[w][lane][j];
                    slots[q] = (unsigned long long)((size_t)(k0 + lane) * cap + (size_t)(b0 + j));
                }
            }
            // every lane's reads of this window are done before the next one is written
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// [begin, end) of every cell's run in the sorted list (cells without records
// keep 0, 0)
__global__ void k_det_bounds(const unsigned *__restrict__ keys, int64_t total, int *begin,
                             int *end)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        const unsigned k = keys[j];
        if (j == 0 || keys[j - 1] != k) begin[k] = (int)j;
        if (j == total - 1 || keys[j + 1] != k) end[k] = (int)(j + 1);
    }
}

// the 16 knot sums of every cell: one wavefront per cell.  Lane 8 r + h
// holds components 2 h, 2 h + 1 and adds the records r, r + 8, ... of the
// cell's run in order, so one load instruction reads eight whole 128-byte
// records; then a fixed butterfly over r.  The order does not depend on
// scheduling.
__global__ void __launch_bounds__(256)
k_det_cellsum(const int *__restrict__ begin, const int *__restrict__ end,
              const unsigned long long *__restrict__ slots, const double *__restrict__ rec,
              int ncell, double *__restrict__ tot)
{
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);   // uniform in the wavefront
    const int lane = threadIdx.x & 63;
    const int r = lane >> 3, h = lane & 7;
    if (c >= ncell) return;
    double t0 = 0.0, t1 = 0.0;
    const int e = end[c];
    int j = begin[c] + r;
    // four records of this lane in flight, added in their order
    for (; j + 24 < e; j += 32) {
        double2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = reinterpret_cast<const double2 *>(rec + (size_t)slots[j + 8 * q] * 16)[h];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            t0 += v[q].x;
            t1 += v[q].y;
        }
    }
    for (; j < e; j += 8) {
        const double2 v = reinterpret_cast<const double2 *>(rec + (size_t)slots[j] * 16)[h];
        t0 += v.x;
        t1 += v.y;
    }
#pragma unroll
    for (int o = 8; o <= 32; o <<= 1) {
        t0 += __shfl_xor(t0, o, 64);
        t1 += __shfl_xor(t1, o, 64);
    }
    if (r == 0) {
        tot[(size_t)(2 * h) * ncell + c] = t0;
        tot[(size_t)(2 * h + 1) * ncell + c] = t1;
    }
}

// dc[r][q] += the entries (kz, kx) of the cells (i2, i1) whose clamped knot
// (clamp(i2 - 1 + kz), clamp(i1 - 1 + kx)) is (r, q), in a fixed order
__global__ void k_det_gather(const double *__restrict__ tot, int n1, int n2, double *dc)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (q >= n1) return;
    const int ncell = (n1 + 8) * (n2 + 8);
    const int i2lo = r == 0 ? -4 : r - 2, i2hi = r == n2 - 1 ? n2 + 3 : r + 1;
    const int i1lo = q == 0 ? -4 : q - 2, i1hi = q == n1 - 1 ? n1 + 3 : q + 1;
    double acc = 0.0;
    for (int i2 = max(i2lo, -4); i2 <= min(i2hi, n2 + 3); ++i2)
        for (int kz = 0; kz < 4; ++kz) {
            if (min(max(i2 - 1 + kz, 0), n2 - 1) != r) continue;
            for (int i1 = max(i1lo, -4); i1 <= min(i1hi, n1 + 3); ++i1)
                for (int kx = 0; kx < 4; ++kx) {
                    if (min(max(i1 - 1 + kx, 0), n1 - 1) != q) continue;
                    acc += tot[(size_t)(4 * kz + kx) * ncell + (i2 + 4) * (n1 + 8) + (i1 + 4)];
                }
        }
    dc[(size_t)r * n1 + q] += acc;
}

// Layout of the log buffer for R slots per beam: records [R][cap][16] doubles,
// cells [R][cap] ints, lengths [cap] ints.
static const int *det_counts(const fga_ctx *ctx, int64_t cap, int R)
{
    return (const int *)((const char *)ctx->det_log + (size_t)R * 16 * cap * sizeof(double) +
                         (size_t)R * cap * sizeof(int));
}

fga_status fga_det_stats(fga_ctx *ctx, const fga_beams *beams, int nshots, int R, int64_t out[3])
{
    const int64_t cap = beams->capacity;
    fga_status rc = fga_ensure(ctx, &ctx->det_cell, &ctx->det_cell_bytes,
                               std::max(ctx->det_cell_bytes, (size_t)4 * sizeof(unsigned long long)),
                               "deterministic reduction workspace");
    if (rc != FGA_OK) return rc;
    unsigned long long *stats = (unsigned long long *)ctx->det_cell;
    const int *cnt = det_counts(ctx, cap, R);
    hipLaunchKernelGGL(k_det_zero_u64, dim3(1), dim3(64), 0, ctx->stream, stats, 4);
    hipLaunchKernelGGL(k_det_stats, dim3(ctx->num_cu * 4), dim3(256), 0, ctx->stream,
                       beams->offsets, nshots, cnt, stats);
    FGA_HIP(ctx, hipGetLastError());
    unsigned long long h[3];
    FGA_HIP(ctx, hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    FGA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out[0] = (int64_t)h[0];
    out[1] = (int64_t)h[1];
    out[2] = (int64_t)h[2];
    return FGA_OK;
}

fga_status fga_det_reduce(fga_ctx *ctx, int64_t cap, int R, int64_t nb, int64_t total,
                          double *dc)
{
    if (total == 0 || nb == 0) return FGA_OK;
    if (total > 2147483647LL)
        return fga_fail(ctx, FGA_EINVAL, "deterministic reduction of %lld records is too large",
                        (long long)total);
    hipStream_t st = ctx->stream;
    const int n1 = ctx->g.n1, n2 = ctx->g.n2;
    const int ncell = (n1 + 8) * (n2 + 8);
    unsigned nbits = 1;
    while (nbits < 32 && (1u << nbits) < (unsigned)ncell) ++nbits;
    const char *lg = (const char *)ctx->det_log;
    const double *rec = (const double *)lg;
    const int *cell = (const int *)(lg + (size_t)R * 16 * cap * sizeof(double));
    const int *cnt = det_counts(ctx, cap, R);

    // workspace: offsets, keys and slots (in and sorted), rocPRIM temporaries
    size_t scan_tmp = 0, sort_tmp = 0;
    FGA_HIP(ctx, rocprim::exclusive_scan(nullptr, scan_tmp, cnt, (int64_t *)nullptr, (int64_t)0,
                                         (size_t)nb, rocprim::plus<int64_t>(), st));
    FGA_HIP(ctx, rocprim::radix_sort_pairs(nullptr, sort_tmp, (const unsigned *)nullptr,
                                           (unsigned *)nullptr,
                                           (const unsigned long long *)nullptr,
                                           (unsigned long long *)nullptr, (size_t)total, 0,
                                           nbits, st));
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_off = al((size_t)nb * sizeof(int64_t));
    const size_t b_keys = al((size_t)total * sizeof(unsigned));
    const size_t b_slots = al((size_t)total * sizeof(unsigned long long));
    const size_t b_tmp = al(std::max(scan_tmp, sort_tmp));
    fga_status rc = fga_ensure(ctx, &ctx->det_sort, &ctx->det_sort_bytes,
                               b_off + 2 * b_keys + 2 * b_slots + b_tmp,
                               "deterministic reduction sort workspace");
    if (rc != FGA_OK) return rc;
    char *w = (char *)ctx->det_sort;
    int64_t *off = (int64_t *)w;
    unsigned *keys = (unsigned *)(w + b_off);
    unsigned *keys_s = (unsigned *)(w + b_off + b_keys);
    unsigned long long *slots = (unsigned long long *)(w + b_off + 2 * b_keys);
    unsigned long long *slots_s = (unsigned long long *)(w + b_off + 2 * b_keys + b_slots);
    void *tmp = w + b_off + 2 * b_keys + 2 * b_slots;

    // cell runs and sums (the stats words sit in the first 32 bytes)
    const size_t c_hdr = 256;
    const size_t c_be = al((size_t)2 * ncell * sizeof(int));
    rc = fga_ensure(ctx, &ctx->det_cell, &ctx->det_cell_bytes,
                    c_hdr + c_be + (size_t)16 * ncell * sizeof(double),
                    "deterministic reduction workspace");
    if (rc != FGA_OK) return rc;
    int *begin = (int *)((char *)ctx->det_cell + c_hdr);
    int *end = begin + ncell;
    double *tot = (double *)((char *)ctx->det_cell + c_hdr + c_be);

    FGA_HIP(ctx, rocprim::exclusive_scan(tmp, scan_tmp, cnt, off, (int64_t)0, (size_t)nb,
                                         rocprim::plus<int64_t>(), st));
    const int blocks = ctx->num_cu * 4;
    const int64_t lb = std::min<int64_t>((nb + 255) / 256, (int64_t)ctx->num_cu * 8);
    hipLaunchKernelGGL(k_det_list, dim3((unsigned)lb), dim3(256), 0, st, cnt, off, cell, nb, cap,
                       keys, slots);
    FGA_HIP(ctx, hipGetLastError());
    FGA_HIP(ctx, rocprim::radix_sort_pairs(tmp, sort_tmp, keys, keys_s, slots, slots_s,
                                           (size_t)total, 0, nbits, st));
    hipLaunchKernelGGL(k_det_zero_i32, dim3(blocks), dim3(256), 0, st, begin, (int64_t)2 * ncell);
    hipLaunchKernelGGL(k_det_bounds, dim3(blocks), dim3(256), 0, st, keys_s, total, begin, end);
    hipLaunchKernelGGL(k_det_cellsum, dim3((ncell + 3) / 4), dim3(256), 0, st, begin, end,
                       slots_s, rec, ncell, tot);
    hipLaunchKernelGGL(k_det_gather, dim3((n1 + 255) / 256, n2), dim3(256), 0, st, tot, n1, n2,
                       dc);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}
