// Beam -> tile binning and the binned mixed-precision splat.
//
// Every beam's truncation box covers a rectangle of 64 x 64 output tiles.
// The beams are binned into one list per (shot, tile), each list in
// ascending beam order, without sorting:
//   1. k_bin_count       one wavefront per chunk of 1024 beams counts, in LDS,
//                        the beams of the chunk that meet every tile;
//   2. k_bin_seg_sums, k_bin_scan_tiles
//                        per tile, an exclusive scan over the chunks (each
//                        chunk's offset inside the tile's list);
//      k_bin_scan_items  a scan over the tiles (list starts) and the split of
//                        every list into work items of equal length (the last
//                        item of a list shorter);
//   3. k_bin_fill        each chunk again, 64 beams at a time: for each tile of
//                        the lanes' union rectangle a ballot ranks the lanes,
//                        so the lists come out in beam order.
// The splat runs one wavefront per work item (the grid is sized for the
// largest possible item count; wavefronts past the device count leave at
// once); every item writes a private partial tile, and the partial tiles of
// one tile are added in item order.  All counts stay on the device
// (graph-capturable), and the result does not depend on scheduling.
#include "splat.h"

#define BIN_WCH 1024             // beams per wavefront chunk
#define BIN_ITEM_MIN 256         // hits per work item, at least
#define BIN_MAX_TILES 8192       // (shot, tile) pairs per call (LDS counters)
#define BIN_SCAN_GROUPS 16       // chunk groups per workgroup in the chunk scan
#define BIN_SEGS 32              // chunk segments (workgroups) per tile column

struct BinItem {
    int64_t start;   // first entry in the list array
    int32_t len;     // entries
    int32_t tile;    // shot * ntiles + tile
};

struct BinArgs {
    const int64_t *id;
    const int64_t *offsets;
    const short4 *box;
    int nshots;
    int64_t per_shot;     // candidates per shot (2 Nq Np)
    int ntile1, ntiles;   // tiles per row, tiles per shot
    int ntiles_total;
    int32_t *wcnt;        // [chunk][ntiles_total]: counts, then offsets
    int64_t *ssum;        // [BIN_SEGS][ntiles_total]: counts per chunk segment
    int64_t *tile_start;  // [ntiles_total + 1]: counts, then list starts
    int32_t *tile_item;   // [ntiles_total + 1]: first item of each tile
    BinItem *items;       // [max_items]
    int64_t *meta;        // [0] hits, [1] items, [2] item length
    int32_t *list;        // beam indices
    int items_target;     // the item length is about hits / items_target
    int tile;             // tile edge (nodes): SP_T, or SP64_T for the FP64 splat
};

__device__ __forceinline__ int bin_nchunks(const BinArgs &B)
{
    const int64_t nb = B.offsets[B.nshots];
    return (int)((nb + BIN_WCH - 1) / BIN_WCH);
}

__device__ __forceinline__ bool box_tiles(const short4 bx, int T, int &t1lo, int &t1hi,
                                          int &t2lo, int &t2hi)
{
    if (bx.x > bx.y || bx.z > bx.w) return false;
    t1lo = bx.x / T;
    t1hi = bx.y / T;
    t2lo = bx.z / T;
    t2hi = bx.w / T;
    return true;
}

// With diff (the host's choice when nshots (nt1 + 1)(nt2 + 1) counters fit)
// a box adds +1 and -1 at the four corners of its tile rectangle in a
// difference array, whose 2-D prefix sums per shot are the tile counts: four
// LDS atomics per beam instead of one per tile it meets (~33 per beam at
// eps = 1/1024).
__global__ void __launch_bounds__(64)
k_bin_count(BinArgs B, int diff)
{
    extern __shared__ int cnt[];
    const int lane = threadIdx.x;
    const int64_t nb = B.offsets[B.nshots];
    const int nused = bin_nchunks(B);
    const int w1 = B.ntile1 + 1, w2 = B.ntiles / B.ntile1 + 1, per = w1 * w2;
    const int ncnt = diff ? B.nshots * per : B.ntiles_total;
    for (int chunk = blockIdx.x; chunk < nused; chunk += gridDim.x) {
        for (int t = lane; t < ncnt; t += 64) cnt[t] = 0;
        __syncthreads();
        for (int r = 0; r < BIN_WCH / 64; ++r) {
            const int64_t b = (int64_t)chunk * BIN_WCH + r * 64 + lane;
            int t1lo, t1hi, t2lo, t2hi;
            if (b < nb && box_tiles(B.box[b], B.tile, t1lo, t1hi, t2lo, t2hi)) {
                const int s = B.nshots == 1 ? 0 : (int)(B.id[b] / B.per_shot);
                if (diff) {
                    int *d = cnt + s * per;
                    atomicAdd(&d[t2lo * w1 + t1lo], 1);
                    atomicAdd(&d[t2lo * w1 + t1hi + 1], -1);
                    atomicAdd(&d[(t2hi + 1) * w1 + t1lo], -1);
                    atomicAdd(&d[(t2hi + 1) * w1 + t1hi + 1], 1);
                } else {
                    for (int t2 = t2lo; t2 <= t2hi; ++t2)
                        for (int t1 = t1lo; t1 <= t1hi; ++t1)
                            atomicAdd(&cnt[s * B.ntiles + t2 * B.ntile1 + t1], 1);
                }
            }
        }
        __syncthreads();
        if (diff) {
            // prefix sums along each row, then along each column
            for (int row = lane; row < B.nshots * w2; row += 64) {
                int acc = 0;
                for (int t1 = 0; t1 < w1; ++t1) {
                    acc += cnt[row * w1 + t1];
                    cnt[row * w1 + t1] = acc;
                }
            }
            __syncthreads();
            for (int col = lane; col < B.nshots * w1; col += 64) {
                const int s = col / w1, t1 = col - s * w1;
                int acc = 0;
                for (int t2 = 0; t2 < w2; ++t2) {
                    acc += cnt[s * per + t2 * w1 + t1];
                    cnt[s * per + t2 * w1 + t1] = acc;
                }
            }
            __syncthreads();
        }
        int32_t *out = B.wcnt + (size_t)chunk * B.ntiles_total;
        for (int t = lane; t < B.ntiles_total; t += 64) {
            if (diff) {
                const int s = t / B.ntiles, tt = t - s * B.ntiles;
                const int t2 = tt / B.ntile1, t1 = tt - t2 * B.ntile1;
                out[t] = cnt[s * per + t2 * w1 + t1];
            } else {
                out[t] = cnt[t];
            }
        }
        __syncthreads();
    }
}

// Exclusive scan over the chunks of every tile, in two launches over a grid
// of (64 tiles) x (BIN_SEGS chunk segments): k_bin_seg_sums sums each
// segment's counts, k_bin_scan_tiles starts each segment from the sum of the
// segments before it.  Inside a workgroup, thread (group g, lane l) owns tile
// 64 blockIdx.x + l and a contiguous part of the segment; the wavefront reads
// 64 consecutive counts per chunk.
struct SegRange {
    int c0, c1;   // this thread's chunks
};

__device__ __forceinline__ SegRange seg_range(const BinArgs &B, int grp)
{
    const int nused = bin_nchunks(B);
    const int seg = (nused + BIN_SEGS - 1) / BIN_SEGS;
    const int s0 = min((int)blockIdx.y * seg, nused), s1 = min(s0 + seg, nused);
    const int per = (s1 - s0 + BIN_SCAN_GROUPS - 1) / BIN_SCAN_GROUPS;
    SegRange r;
    r.c0 = min(s0 + grp * per, s1);
    r.c1 = min(r.c0 + per, s1);
    return r;
}

__device__ __forceinline__ int64_t col_sum(const int32_t *col, size_t ld, int c0, int c1)
{
    int64_t sum = 0;
    for (int c = c0; c < c1; c += 8) {
        int32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = c + k < c1 ? col[(size_t)(c + k) * ld] : 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += v[k];
    }
    return sum;
}

__global__ void __launch_bounds__(64 * BIN_SCAN_GROUPS)
k_bin_seg_sums(BinArgs B)
{
    __shared__ int64_t gsum[BIN_SCAN_GROUPS][64];
    const int l = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + l;
    const bool ok = t < B.ntiles_total;
    const SegRange r = seg_range(B, grp);
    gsum[grp][l] = ok ? col_sum(B.wcnt + t, (size_t)B.ntiles_total, r.c0, r.c1) : 0;
    __syncthreads();
    if (grp == 0 && ok) {
        int64_t sum = 0;
        for (int k = 0; k < BIN_SCAN_GROUPS; ++k) sum += gsum[k][l];
        B.ssum[(size_t)blockIdx.y * B.ntiles_total + t] = sum;
    }
}

__global__ void __launch_bounds__(64 * BIN_SCAN_GROUPS)
k_bin_scan_tiles(BinArgs B)
{
    __shared__ int64_t gsum[BIN_SCAN_GROUPS][64];
    const int l = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + l;
    const bool ok = t < B.ntiles_total;
    const SegRange r = seg_range(B, grp);
    int32_t *col = B.wcnt + t;
    const size_t ld = (size_t)B.ntiles_total;
    gsum[grp][l] = ok ? col_sum(col, ld, r.c0, r.c1) : 0;
    __syncthreads();
    int64_t run = 0;
    if (ok) {
        for (int y = 0; y < (int)blockIdx.y; ++y) run += B.ssum[(size_t)y * ld + t];
        for (int k = 0; k < grp; ++k) run += gsum[k][l];
        for (int c = r.c0; c < r.c1; c += 8) {
            int32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = c + k < r.c1 ? col[(size_t)(c + k) * ld] : 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (c + k < r.c1) col[(size_t)(c + k) * ld] = (int32_t)run;
                run += v[k];
            }
        }
        // the tile's count, from the last segment's last group
        if (blockIdx.y == BIN_SEGS - 1 && grp == BIN_SCAN_GROUPS - 1) B.tile_start[t] = run;
    }
}

// block-wide exclusive scan of v over 1024 threads; returns the total
__device__ int64_t block_scan_1024(int64_t &v, int64_t *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t x = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const int64_t total = sh[1023];
    v = sh[t] - v;
    __syncthreads();
    return total;
}

#define BIN_PER_THREAD (BIN_MAX_TILES / 1024)

__global__ void __launch_bounds__(1024)
k_bin_scan_items(BinArgs B)
{
    __shared__ int64_t sh[1024];
    __shared__ int32_t s_item[BIN_MAX_TILES + 1];   // first item of every tile
    const int t = threadIdx.x;
    const int T = B.ntiles_total;
    const int lo = t * BIN_PER_THREAD;
    int64_t cnt[BIN_PER_THREAD];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < BIN_PER_THREAD; ++k) {
        cnt[k] = lo + k < T ? B.tile_start[lo + k] : 0;
        sum += cnt[k];
    }
    int64_t off = sum;
    const int64_t H = block_scan_1024(off, sh);
    int64_t L = (H + B.items_target - 1) / B.items_target;
    L = L < BIN_ITEM_MIN ? BIN_ITEM_MIN : (L + 63) / 64 * 64;
    int64_t nit = 0;
#pragma unroll
    for (int k = 0; k < BIN_PER_THREAD; ++k) nit += (cnt[k] + L - 1) / L;
    int64_t ioff = nit;
    const int64_t NI = block_scan_1024(ioff, sh);
    if (t == 0) {
        B.meta[0] = H;
        B.meta[1] = NI;
        B.meta[2] = L;
        B.tile_start[T] = H;
        B.tile_item[T] = (int32_t)NI;
        s_item[T] = (int32_t)NI;
    }
#pragma unroll
    for (int k = 0; k < BIN_PER_THREAD; ++k) {
        if (lo + k >= T) break;
        B.tile_start[lo + k] = off;
        B.tile_item[lo + k] = (int32_t)ioff;
        s_item[lo + k] = (int32_t)ioff;
        ioff += (cnt[k] + L - 1) / L;
        off += cnt[k];
    }
    __syncthreads();
    // the work items, all threads at once: item i belongs to the tile k with
    // s_item[k] <= i < s_item[k + 1] (tiles without items never satisfy it)
    for (int i = t; i < (int)NI; i += 1024) {
        int a = 0, b = T;
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (s_item[m] <= i) a = m;
            else b = m;
        }
        const int64_t e = (int64_t)(i - s_item[a]) * L;
        const int64_t n = B.tile_start[a + 1] - B.tile_start[a];
        BinItem it;
        it.start = B.tile_start[a] + e;
        it.len = (int32_t)(n - e < L ? n - e : L);
        it.tile = a;
        B.items[i] = it;
    }
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__global__ void __launch_bounds__(64)
k_bin_fill(BinArgs B)
{
    // next list position of every shot-tile for this chunk: its list start
    // plus the entries of the chunks before, advanced as entries are written
    extern __shared__ int64_t pos[];
    const int lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nb = B.offsets[B.nshots];
    const int nused = bin_nchunks(B);
    for (int chunk = blockIdx.x; chunk < nused; chunk += gridDim.x) {
        const int32_t *woff = B.wcnt + (size_t)chunk * B.ntiles_total;
        for (int t = lane; t < B.ntiles_total; t += 64) pos[t] = B.tile_start[t] + woff[t];
        __syncthreads();
        for (int r = 0; r < BIN_WCH / 64; ++r) {
            const int64_t b = (int64_t)chunk * BIN_WCH + r * 64 + lane;
            int t1lo = 0, t1hi = -1, t2lo = 0, t2hi = -1, s = -1;
            if (b < nb && box_tiles(B.box[b], B.tile, t1lo, t1hi, t2lo, t2hi))
                s = B.nshots == 1 ? 0 : (int)(B.id[b] / B.per_shot);
            const int smin = wave_min(s < 0 ? 0x7fffffff : s), smax = wave_max(s);
            for (int ss = smin; ss <= smax; ++ss) {
                const bool mine = s == ss;
                if (!__ballot(mine)) continue;
                const int u1lo = wave_min(mine ? t1lo : 0x7fffffff);
                const int u1hi = wave_max(mine ? t1hi : -1);
                const int u2lo = wave_min(mine ? t2lo : 0x7fffffff);
                const int u2hi = wave_max(mine ? t2hi : -1);
                for (int t2 = u2lo; t2 <= u2hi; ++t2)
                    for (int t1 = u1lo; t1 <= u1hi; ++t1) {
                        const bool hit =
                            mine && t1 >= t1lo && t1 <= t1hi && t2 >= t2lo && t2 <= t2hi;
                        const unsigned long long m = __ballot(hit);
                        if (!m) continue;
                        const int tt = ss * B.ntiles + t2 * B.ntile1 + t1;
                        const int64_t base = pos[tt];
                        if (hit) B.list[base + __popcll(m & below)] = (int32_t)b;
                        __builtin_amdgcn_wave_barrier();
                        if (lane == 0) pos[tt] = base + __popcll(m);
                        __builtin_amdgcn_wave_barrier();
                    }
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_splat_binned(SplatArgs A, BinArgs B, const SplatRec *__restrict__ rec)
{
    // records of the current 64 list entries; wavefront-private, read back
    // with uniform addresses
    __shared__ SplatRec stage_rec[4][64];
    SplatRec *st = stage_rec[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    // the item index is uniform over the wavefront: keep it (and with it the
    // tile origin, the list range and every block test) in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const float hl2e = (float)A.half_inv_eps * 1.4426950408889634f;
    // whole wavefronts leave; no workgroup barrier below
    if (it < (int)B.meta[1]) {
        const BinItem item = B.items[it];
        const int t = item.tile % B.ntiles;
        const int X0 = (t % A.ntile1) * SP_T, Z0 = (t / A.ntile1) * SP_T;
        const int i1 = X0 + lane, i2 = Z0 + lane;
        const double x1 = A.o1 + i1 * A.d1, x2 = A.o2 + i2 * A.d2;
        floatx16 acc00, acc01, acc10, acc11;
        double acc64[4][16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc00[r] = acc01[r] = acc10[r] = acc11[r] = 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc64[q][r] = 0.0;
        }
        const int32_t *lst = B.list + item.start;
        int32_t b_next = lane < item.len ? lst[lane] : 0;
        int chunks = 0;
        for (int k0 = 0; k0 < item.len; k0 += 64) {
            const int nk = min(64, item.len - k0);
            const int32_t b = b_next;
            if (k0 + 64 + lane < item.len) b_next = lst[k0 + 64 + lane];
            if (lane < nk) {
                const float4 *src = reinterpret_cast<const float4 *>(rec + b);
                float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
                float4 *dst = reinterpret_cast<float4 *>(st + lane);
                dst[0] = q0;
                dst[1] = q1;
                dst[2] = q2;
                dst[3] = q3;
            }
            __builtin_amdgcn_wave_barrier();
            // software pipeline: the next record is read and its factors
            // formed while the matrix cores work on the current beam
            SplatRec r = st[0];
            Frags fr = beam_frags(r, i1, i2, x1, x2, hl2e);
            for (int k = 1; k < nk; ++k) {
                SplatRec rn = st[k];
                tile_update(fr, acc00, acc01, acc10, acc11);
                r = rn;
                fr = beam_frags(r, i1, i2, x1, x2, hl2e);
            }
            tile_update(fr, acc00, acc01, acc10, acc11);
            __builtin_amdgcn_wave_barrier();
            // fold the FP32 sums (256 beams at most) into FP64
            if (++chunks == 4) {
                chunks = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    acc64[0][k] += (double)acc00[k];
                    acc64[1][k] += (double)acc01[k];
                    acc64[2][k] += (double)acc10[k];
                    acc64[3][k] += (double)acc11[k];
                    acc00[k] = acc01[k] = acc10[k] = acc11[k] = 0.f;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            acc64[0][k] += (double)acc00[k];
            acc64[1][k] += (double)acc01[k];
            acc64[2][k] += (double)acc10[k];
            acc64[3][k] += (double)acc11[k];
        }
        // D[i][j] of a 32 x 32 block: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4;
        // block (a, c) covers tile rows 32 a + i and tile columns 32 c + j
        double *out = A.partial + (size_t)it * SP_T * SP_T;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int row = 32 * (q >> 1) + 8 * (k >> 2) + 4 * (lane >> 5) + (k & 3);
                const int col = 32 * (q & 1) + (lane & 31);
                out[row * SP_T + col] = acc64[q][k];
            }
    }
}

// The binned splat with FP16 hi/lo split products (FGA_MIXED_SPLIT): the
// same work items, records and partial tiles as k_splat_binned; the beams of
// an item are taken two at a time, the lower half of the wavefront forming
// the factors of the first and the upper half those of the second (an odd
// last beam pairs with a staged record of weight zero).  U is scaled by 2^ks
// per shot with max |C a| 2^ks < 2^14, and the FP64 fold multiplies by 2^-ks
// (exact).  Staging a chunk, lane k forms what beam k needs beyond its
// record: the scaled |C a| and its 32-node rotations (SplitRec).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_splat_binned_split(SplatArgs A, BinArgs B, const SplatRec *__restrict__ rec)
{
    __shared__ SplitRec stage_rec[4][64];
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, li = lane & 31;
    const int it = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    // Gaussian coordinates: exp(-r^2 / (2 eps)) = exp2(-(r sqh)^2)
    const double sqh = sqrt(A.half_inv_eps * 1.4426950408889634);
    if (it < (int)B.meta[1]) {
        const BinItem item = B.items[it];
        const int shot = item.tile / B.ntiles;
        const int t = item.tile % B.ntiles;
        const int X0 = (t % A.ntile1) * SP_T, Z0 = (t / A.ntile1) * SP_T;
        const double x1 = A.o1 + (X0 + li) * A.d1, x2 = A.o2 + (Z0 + li) * A.d2;
        const double xs1 = x1 * sqh, xs2 = x2 * sqh;
        const double d32_1 = 32.0 * A.d1, d32_2 = 32.0 * A.d2;
        const float d32s_1 = (float)(d32_1 * sqh), d32s_2 = (float)(d32_2 * sqh);
        // the shot's power of two
        const float wm = __uint_as_float(A.wmax[shot]);
        int ks = 0;
        if (wm > 0.f && wm <= 3.0e38f) {
            int e;
            (void)frexpf(wm, &e);      // wm < 2^e
            ks = 14 - e;
        }
        const float wsc = ldexpf(1.f, ks);
        const double inv = ldexp(1.0, -ks);
        floatx16 acc00, acc01, acc10, acc11;
        double acc64[4][16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc00[r] = acc01[r] = acc10[r] = acc11[r] = 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc64[q][r] = 0.0;
        }
        const int32_t *lst = B.list + item.start;
        int32_t b_next = lane < item.len ? lst[lane] : 0;
        int chunks = 0;
        for (int k0 = 0; k0 < item.len; k0 += 64) {
            const int nk = min(64, item.len - k0);
            const int32_t b = b_next;
            if (k0 + 64 + lane < item.len) b_next = lst[k0 + 64 + lane];
            if (lane < nk) {
                const SplatRec r = rec[b];
                SplitRec sr;
                sr.A1 = r.A1;
                sr.B1 = r.B1;
                sr.A2 = r.A2;
                sr.B2 = r.B2;
                sr.Q1s = r.Q1 * sqh;
                sr.Q2s = r.Q2 * sqh;
                sr.w = r.w * wsc;
                const double t1 = r.B1 * d32_1, t2 = r.B2 * d32_2;
                const float th1 = (float)(t1 - rint(t1)), th2 = (float)(t2 - rint(t2));
                sr.r1c = __builtin_amdgcn_cosf(th1);
                sr.r1s = __builtin_amdgcn_sinf(th1);
                sr.r2c = __builtin_amdgcn_cosf(th2);
                sr.r2s = __builtin_amdgcn_sinf(th2);
                sr.pad[0] = sr.pad[1] = sr.pad[2] = 0.f;
                stage_rec[wv][lane] = sr;
            } else if (lane == nk) {
                // an odd chunk's partner of its last beam: zero weight, finite factors
                SplitRec z;
                z.A1 = z.B1 = z.A2 = z.B2 = z.Q1s = z.Q2s = 0.0;
                z.w = z.r1s = z.r2s = 0.f;
                z.r1c = z.r2c = 1.f;
                z.pad[0] = z.pad[1] = z.pad[2] = 0.f;
                stage_rec[wv][lane] = z;
            }
            __builtin_amdgcn_wave_barrier();
            // beam 2 p + h of the chunk in this half
            const int npair = (nk + 1) >> 1;
            for (int pp = 0; pp < npair; ++pp) {
                const SplitRec r = stage_rec[wv][2 * pp + h];
                const SplitFrags fr = beam_split(r, r.w, x1, x2, xs1, xs2, d32s_1, d32s_2);
                tile_update_split(fr, acc00, acc01, acc10, acc11);
            }
            __builtin_amdgcn_wave_barrier();
            // fold the FP32 sums (256 beams at most) into FP64
            if (++chunks == 4) {
                chunks = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    acc64[0][k] += (double)acc00[k] * inv;
                    acc64[1][k] += (double)acc01[k] * inv;
                    acc64[2][k] += (double)acc10[k] * inv;
                    acc64[3][k] += (double)acc11[k] * inv;
                    acc00[k] = acc01[k] = acc10[k] = acc11[k] = 0.f;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            acc64[0][k] += (double)acc00[k] * inv;
            acc64[1][k] += (double)acc01[k] * inv;
            acc64[2][k] += (double)acc10[k] * inv;
            acc64[3][k] += (double)acc11[k] * inv;
        }
        double *out = A.partial + (size_t)it * SP_T * SP_T;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int row = 32 * (q >> 1) + 8 * (k >> 2) + 4 * (lane >> 5) + (k & 3);
                const int col = 32 * (q & 1) + (lane & 31);
                out[row * SP_T + col] = acc64[q][k];
            }
    }
}

// The binned FP64 splat: one workgroup per work item (a tile of SP64_T x
// SP64_T nodes and a run of its list); every listed beam meets the tile, so
// the factor batches are full (16 beams) and nothing is scanned.  The
// factors are staged as in k_splat64 (V conjugated), and the sum runs on
// the FP64 matrix cores: wavefront w owns the 64 x 64 quadrant
// (x1 from X0 + 64 (w & 1), x2 from Z0 + 64 (w >> 1)), 4 x 4 blocks of
// 16 x 16, and the beams are taken two at a time,
//   u[x1][x2] += sum_k A[x1][k] B[k][x2],  k = (beam of the pair, re / im),
//   A = [Re U, Im U],  B = [Re conj V ; Im conj V] = [Re V ; -Im V],
// one v_mfma_f64_16x16x4f64 per block (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element i of its result is D[4 i + l / 16][l % 16]).
// A and B are read from the staged factors as they are: no vector FP64
// work in the loop (the matrix cores and the FP64 vector instructions share
// one pipe).  An odd batch pairs its last beam with a slot staged as zero.
// The item's partial tile goes to its own slot for k_splat_reduce_binned.
typedef double sp64x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_splat64_binned(SplatArgs A, BinArgs B)
{
    __shared__ double2 U[SP64_KC][SP64_T];
    __shared__ double2 Vf[SP64_KC][SP64_T];
    const int it = blockIdx.x;
    if (it >= (int)B.meta[1]) return;            // the grid covers the most items there can be
    const BinItem item = B.items[it];
    const int tl = item.tile % B.ntiles;
    const int X0 = (tl % A.ntile1) * SP64_T, Z0 = (tl / A.ntile1) * SP64_T;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int q1 = 64 * (w & 1), q2 = 64 * (w >> 1);
    const int mrow = lane & 15, pb = lane >> 5, part = (lane >> 4) & 1;
    const double kap1 = exp(-A.d1 * A.d1 * A.inv_eps), kap2 = exp(-A.d2 * A.d2 * A.inv_eps);
    sp64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = sp64x4{0.0, 0.0, 0.0, 0.0};
    const int32_t *lst = B.list + item.start;
    for (int k0 = 0; k0 < item.len; k0 += SP64_KC) {
        const int k = t >> 4;
        sp64_stage<true>(A, k0 + k < item.len ? (int64_t)lst[k0 + k] : -1, X0, Z0, t & 15, kap1,
                         kap2, U[k], Vf[k]);
        __syncthreads();
        const int kn = min(SP64_KC, item.len - k0);
        for (int p = 0; p < kn; p += 2) {
            // this lane's beam of the pair and part: slot p + pb (staged as
            // zero past the batch), component part of the stored pair
            const double *ua = reinterpret_cast<const double *>(&U[p + pb][q1 + mrow]) + part;
            const double *vb = reinterpret_cast<const double *>(&Vf[p + pb][q2 + mrow]) + part;
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = ua[32 * a];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = vb[32 * c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0,
                                                                     0, 0);
        }
        __syncthreads();
    }
    // element i of block (a, c): x1 = q1 + 16 a + 4 i + lane / 16, x2 = q2 + 16 c + lane % 16
    double *out = A.partial + (size_t)it * SP64_T * SP64_T;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[(q2 + 16 * c + mrow) * SP64_T + q1 + 16 * a + 4 * i + (lane >> 4)] =
                    acc[a][c][i];
}

// u[s][i2][i1] = the sum of the partial tiles of its tile, in item order
__global__ void k_splat_reduce_binned(SplatArgs A, BinArgs B, double *__restrict__ u)
{
    const int64_t npts = (int64_t)A.n1 * A.n2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts * B.nshots;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(i / npts);
        const int64_t x = i - s * npts;
        const int i2 = (int)(x / A.n1), i1 = (int)(x - (int64_t)i2 * A.n1);
        const int T = B.tile;
        const size_t T2 = (size_t)T * T;
        const int tt = s * B.ntiles + (i2 / T) * A.ntile1 + i1 / T;
        const int local = (i2 % T) * T + (i1 % T);
        const int a = B.tile_item[tt], e = B.tile_item[tt + 1];
        const double *p = A.partial + local;
        double v = 0.0;
        int it = a;
        // eight loads in flight, added in item order as one at a time would
        for (; it + 8 <= e; it += 8) {
            double w[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) w[q] = p[(size_t)(it + q) * T2];
#pragma unroll
            for (int q = 0; q < 8; ++q) v += w[q];
        }
        for (; it < e; ++it) v += p[(size_t)it * T2];
        u[i] = v;
    }
}

bool fga_splat_binned_fits(const fga_ctx *ctx, int nshots, int T)
{
    const int64_t nt1 = (ctx->g.n1 + T - 1) / T, nt2 = (ctx->g.n2 + T - 1) / T;
    return nt1 * nt2 * nshots <= BIN_MAX_TILES;
}

// Launches the binned splat of the boxes k_splat_prep wrote, on tiles of
// edge `edge`: SP_T for the mixed splats (which also read its records), SP64_T
// for the FP64 one (which reads the beams).
fga_status fga_launch_splat_binned(fga_ctx *ctx, const fga_beams *beams, int nshots, double *u,
                                   SplatArgs A, const void *rec, const void *box, int edge)
{
    const fga_grid &g = ctx->g;
    const int nt1 = (g.n1 + edge - 1) / edge, nt2 = (g.n2 + edge - 1) / edge;
    const int ntiles = nt1 * nt2;
    const int T = ntiles * nshots;
    if (T > BIN_MAX_TILES)
        return fga_fail(ctx, FGA_EINVAL, "binned splat: %d tiles exceed %d", T, BIN_MAX_TILES);
    const int64_t cap = beams->capacity;
    const int64_t nchunks = (cap + BIN_WCH - 1) / BIN_WCH;
    // tiles one box can meet along each axis (a box is 2 Rw + 1 nodes wide)
    const int64_t tp1 = std::min<int64_t>(nt1, 2 * ctx->Rw1 / edge + 2);
    const int64_t tp2 = std::min<int64_t>(nt2, 2 * ctx->Rw2 / edge + 2);
    // one wavefront (FP64: one workgroup of four) per item: about units per
    // CU, set by the autotuner (32 by default: at large2048 the FP64 splat
    // takes 1.73 s with 4 and 1.36 s with 32, the last round of long items
    // shorter).  The sum over tiles of ceil(count / L) is at most
    // hits / L + tiles, and hits / L <= items_target.
    const bool fp64 = edge == SP64_T;
    const int units = ctx->splat_units_per_cu > 0 ? ctx->splat_units_per_cu : 32;
    const int items_target = units * ctx->num_cu;
    const int max_items = items_target + T;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_wcnt = take((size_t)nchunks * T * sizeof(int32_t));
    const size_t o_ssum = take((size_t)BIN_SEGS * T * sizeof(int64_t));
    const size_t o_ts = take((size_t)(T + 1) * sizeof(int64_t));
    const size_t o_ti = take((size_t)(T + 1) * sizeof(int32_t));
    const size_t o_items = take((size_t)max_items * sizeof(BinItem));
    const size_t o_meta = take(4 * sizeof(int64_t));
    const size_t o_list = take((size_t)cap * tp1 * tp2 * sizeof(int32_t));
    fga_status rc = fga_ensure(ctx, &ctx->bin, &ctx->bin_bytes, off, "binning workspace");
    if (rc != FGA_OK) return rc;
    rc = fga_ensure(ctx, (void **)&ctx->partial, &ctx->partial_bytes,
                    (size_t)max_items * edge * edge * sizeof(double), "splat partials");
    if (rc != FGA_OK) return rc;
    char *w = (char *)ctx->bin;
    BinArgs B;
    B.id = beams->id;
    B.offsets = beams->offsets;
    B.box = (const short4 *)box;
    B.nshots = nshots;
    B.per_shot = 2LL * ctx->p.nq1 * ctx->p.nq2 * ctx->p.np1 * ctx->p.np2;
    B.ntile1 = nt1;
    B.ntiles = ntiles;
    B.ntiles_total = T;
    B.wcnt = (int32_t *)(w + o_wcnt);
    B.ssum = (int64_t *)(w + o_ssum);
    B.tile_start = (int64_t *)(w + o_ts);
    B.tile_item = (int32_t *)(w + o_ti);
    B.items = (BinItem *)(w + o_items);
    B.meta = (int64_t *)(w + o_meta);
    B.list = (int32_t *)(w + o_list);
    B.items_target = items_target;
    B.tile = edge;
    A.partial = ctx->partial;
    A.ntile1 = nt1;
    A.tile = edge;
    const int ndiff = nshots * (nt1 + 1) * (nt2 + 1);
    const int diff = ndiff <= BIN_MAX_TILES;
    const size_t lds = (size_t)(diff ? ndiff : T) * sizeof(int);
    const int cgrid = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks, 16 * ctx->num_cu));
    hipLaunchKernelGGL(k_bin_count, dim3(cgrid), dim3(64), lds, ctx->stream, B, diff);
    hipLaunchKernelGGL(k_bin_seg_sums, dim3((T + 63) / 64, BIN_SEGS), dim3(64 * BIN_SCAN_GROUPS),
                       0, ctx->stream, B);
    hipLaunchKernelGGL(k_bin_scan_tiles, dim3((T + 63) / 64, BIN_SEGS),
                       dim3(64 * BIN_SCAN_GROUPS), 0, ctx->stream, B);
    hipLaunchKernelGGL(k_bin_scan_items, dim3(1), dim3(1024), 0, ctx->stream, B);
    hipLaunchKernelGGL(k_bin_fill, dim3(cgrid), dim3(64), (size_t)T * sizeof(int64_t),
                       ctx->stream, B);
    if (fp64)
        hipLaunchKernelGGL(k_splat64_binned, dim3(max_items), dim3(256), 0, ctx->stream, A, B);
    else if (A.wmax)
        hipLaunchKernelGGL(k_splat_binned_split, dim3((max_items + 3) / 4), dim3(256), 0,
                           ctx->stream, A, B, (const SplatRec *)rec);
    else
        hipLaunchKernelGGL(k_splat_binned, dim3((max_items + 3) / 4), dim3(256), 0, ctx->stream,
                           A, B, (const SplatRec *)rec);
    hipLaunchKernelGGL(k_splat_reduce_binned, dim3(1024), dim3(256), 0, ctx->stream, A, B, u);
    FGA_HIP(ctx, hipGetLastError());
    return FGA_OK;
}
