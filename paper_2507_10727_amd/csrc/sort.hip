// Cell sort with compaction: a counting sort of live particles by cell
// (bin = j * nr + i, row-major) into the second particle buffer.  Absorbed
// slots (key < 0) are dropped, so the sort also compacts.
//
// Sorted particles let a chunk of consecutive slots touch only a small box
// of nodes (LDS deposit tiles, cache-local gathers).  Between sorts the
// particles drift, so the array is only nearly sorted: each block takes
// chunks of SORT_CHUNK consecutive slots and counts their bins in LDS over a
// window of SORT_WIN bins starting at the chunk's lowest bin, then issues one
// global atomic per bin of the window (histogram: add the count; scatter:
// reserve the chunk's range of the bin and rank its particles in LDS).
// Bins outside the window (new particles appended at the end, far jumps)
// take one global atomic per wavefront run of equal bins.
#include "common.h"

namespace pic {

namespace {

constexpr int SCAN_TILE = 1024;

// Run structure of the wavefront: lanes with the same valid bin that are
// adjacent form a run; returns the run's first lane and length.
__device__ __forceinline__ void wave_runs(int bin, bool valid, int lane, int &head, int &len)
{
    const int prev = __shfl_up(bin, 1, 64);
    const int pvalid = __shfl_up((int)valid, 1, 64);
    const bool is_head = valid && (lane == 0 || !pvalid || prev != bin);
    const unsigned long long heads = __ballot(is_head);
    const unsigned long long bounds = heads | __ballot(!valid);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const unsigned long long h = heads & upto;
    head = h ? 63 - __clzll(h) : lane;
    const unsigned long long above = bounds & ~upto;
    const int nxt = above ? (__ffsll((long long)above) - 1) : 64;
    len = nxt - head;
}

// Bin (cell j * nr + i) of slot p, -1 if absorbed.
template <typename T>
__device__ __forceinline__ int sort_bin(const SpeciesDev<T> &S, int64_t p, int32_t nr)
{
    if constexpr (sizeof(T) == 4) {
        const int32_t wz = ((const int32_t *)S.fz)[p];
        if (wz < 0) return -1;
        return pos_cell((uint32_t)wz) * nr + pos_cell(((const uint32_t *)S.fr)[p]);
    } else {
        const int k = S.key[p];
        return k >= 0 ? (k >> 16) * nr + (k & 0xffff) : -1;
    }
}

constexpr int SORT_CHUNK = 4096;              // slots per block and chunk (16 per thread)
constexpr int SORT_PER_THREAD = SORT_CHUNK / 256;
constexpr int SORT_WIN = 4096;                // LDS bins per chunk

// Lowest valid bin of the chunk (all threads; INT_MAX if none).  Ends with
// a barrier.
__device__ __forceinline__ int chunk_min_bin(const int *bins, int *red)
{
    int mn = 0x7fffffff;
#pragma unroll
    for (int m = 0; m < SORT_PER_THREAD; ++m)
        if (bins[m] >= 0) mn = min(mn, bins[m]);
    mn = wave_min(mn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
    __syncthreads();
    return min(min(red[0], red[1]), min(red[2], red[3]));
}

template <typename T>
__device__ __forceinline__ void sort_hist_body(const SpeciesDev<T> &S, const DevScalars *sc,
                                               int species, int32_t nr, int32_t *hist, int bid,
                                               int nb)
{
    __shared__ int cnt[SORT_WIN];
    __shared__ int red[4];
    const int64_t n = sc->count[species];
    const int lane = threadIdx.x & 63;
    for (int q = threadIdx.x; q < SORT_WIN; q += 256) cnt[q] = 0;
    for (int64_t base = (int64_t)bid * SORT_CHUNK; base < n; base += (int64_t)nb * SORT_CHUNK) {
        int bins[SORT_PER_THREAD];
#pragma unroll
        for (int m = 0; m < SORT_PER_THREAD; ++m) {
            const int64_t p = base + m * 256 + threadIdx.x;
            bins[m] = (p < n) ? sort_bin(S, p, nr) : -1;
        }
        const int w0 = chunk_min_bin(bins, red);       // (barrier: cnt is zero)
#pragma unroll
        for (int m = 0; m < SORT_PER_THREAD; ++m) {
            const bool valid = bins[m] >= 0;
            int head, len;
            wave_runs(bins[m], valid, lane, head, len);
            if (valid && head == lane) {
                const int w = bins[m] - w0;
                if (w < SORT_WIN) atomicAdd(&cnt[w], len);
                else atomicAdd(&hist[bins[m]], len);
            }
        }
        __syncthreads();
        // flush the window and leave it zero for the next chunk
        for (int q = threadIdx.x; q < SORT_WIN; q += 256) {
            const int c = cnt[q];
            if (c) {
                atomicAdd(&hist[w0 + q], c);
                cnt[q] = 0;
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_sort_hist(SpeciesDev<T> S, const DevScalars *sc,
                                                    int species, int32_t nr, int32_t *hist)
{
    sort_hist_body(S, sc, species, nr, hist, (int)blockIdx.x, (int)gridDim.x);
}

// Exclusive scan of hist[0, nbins) in three passes (tile sums, scan of the
// tile sums in one block, tile scans with offsets).
__device__ __forceinline__ void scan_tiles_body(const int32_t *in, int32_t nbins,
                                                int32_t *tile_sums, int tile)
{
    __shared__ int32_t part[SCAN_TILE / 64];
    const int t0 = tile * SCAN_TILE;
    int v = 0;
    for (int q = threadIdx.x; q < SCAN_TILE; q += blockDim.x) {
        const int b = t0 + q;
        if (b < nbins) v += in[b];
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) s += part[w];
        tile_sums[tile] = s;
    }
}

__global__ void k_scan_tiles(const int32_t *in, int32_t nbins, int32_t *tile_sums)
{
    scan_tiles_body(in, nbins, tile_sums, (int)blockIdx.x);
}

__device__ __forceinline__ void scan_top_body(int32_t *tile_sums, int32_t ntiles, DevScalars *sc,
                                              int species)
{
    // one block of 1024 threads, ntiles <= 1024 * 64 handled by a serial loop per thread
    __shared__ int32_t buf[1024];
    const int per = (ntiles + 1023) / 1024;
    const int start = threadIdx.x * per;
    int local = 0;
    for (int q = 0; q < per; ++q) {
        const int t = start + q;
        if (t < ntiles) local += tile_sums[t];
    }
    buf[threadIdx.x] = local;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = (threadIdx.x >= (unsigned)o) ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += v;
        __syncthreads();
    }
    int run = buf[threadIdx.x] - local;   // exclusive prefix of this thread
    for (int q = 0; q < per; ++q) {
        const int t = start + q;
        if (t < ntiles) {
            const int v = tile_sums[t];
            tile_sums[t] = run;
            run += v;
        }
    }
    if (threadIdx.x == 1023) sc->sort_total[species] = buf[1023];
}

__global__ void k_scan_top(int32_t *tile_sums, int32_t ntiles, DevScalars *sc, int species)
{
    scan_top_body(tile_sums, ntiles, sc, species);
}

__device__ __forceinline__ void scan_down_body(int32_t *data, int32_t nbins,
                                               const int32_t *tile_offsets, int tile)
{
    // one block of SCAN_TILE threads per tile
    __shared__ int32_t buf[SCAN_TILE];
    const int b = tile * SCAN_TILE + threadIdx.x;
    const int v = (b < nbins) ? data[b] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_TILE; o <<= 1) {
        const int a = (threadIdx.x >= (unsigned)o) ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += a;
        __syncthreads();
    }
    if (b < nbins) data[b] = tile_offsets[tile] + buf[threadIdx.x] - v;
}

__global__ void k_scan_down(int32_t *data, int32_t nbins, const int32_t *tile_offsets)
{
    scan_down_body(data, nbins, tile_offsets, (int)blockIdx.x);
}

template <typename T>
__device__ __forceinline__ void copy_slot(const SpeciesDev<T> &src, const SpeciesDev<T> &dst,
                                          int64_t p, int64_t d)
{
    if constexpr (sizeof(T) == 4) {
        // packed position words, copied as bits
        ((uint32_t *)dst.fr)[d] = ((const uint32_t *)src.fr)[p];
        ((uint32_t *)dst.fz)[d] = ((const uint32_t *)src.fz)[p];
    } else {
        dst.key[d] = src.key[p];
        dst.fr[d] = src.fr[p];
        dst.fz[d] = src.fz[p];
    }
    dst.vr[d] = src.vr[p];
    dst.vt[d] = src.vt[p];
    dst.vz[d] = src.vz[p];
    dst.id[d] = src.id[p];
}

template <typename T>
__device__ __forceinline__ void sort_scatter_body(const SpeciesDev<T> &src,
                                                  const SpeciesDev<T> &dst, const DevScalars *sc,
                                                  int species, int32_t nr, int32_t *off, int bid,
                                                  int nb)
{
    __shared__ int cnt[SORT_WIN];     // counts, then the chunk's first slot per bin
    __shared__ int rk[SORT_WIN];      // slots of the bin handed out so far
    __shared__ int red[4];
    const int64_t n = sc->count[species];
    const int lane = threadIdx.x & 63;
    for (int q = threadIdx.x; q < SORT_WIN; q += 256) cnt[q] = 0;
    for (int64_t base = (int64_t)bid * SORT_CHUNK; base < n; base += (int64_t)nb * SORT_CHUNK) {
        int bins[SORT_PER_THREAD];
        uint32_t wr[SORT_PER_THREAD], wz[SORT_PER_THREAD];   // FP32: the position words
#pragma unroll
        for (int m = 0; m < SORT_PER_THREAD; ++m) {
            const int64_t p = base + m * 256 + threadIdx.x;
            if constexpr (sizeof(T) == 4) {
                wr[m] = 0u;
                wz[m] = 0xFFFFFFFFu;
                if (p < n) {
                    wr[m] = ((const uint32_t *)src.fr)[p];
                    wz[m] = ((const uint32_t *)src.fz)[p];
                }
                bins[m] = ((int32_t)wz[m] < 0) ? -1 : pos_cell(wz[m]) * nr + pos_cell(wr[m]);
            } else {
                bins[m] = (p < n) ? sort_bin(src, p, nr) : -1;
            }
        }
        const int w0 = chunk_min_bin(bins, red);       // (barrier: cnt is zero)
        // count the window's bins
#pragma unroll
        for (int m = 0; m < SORT_PER_THREAD; ++m) {
            const bool valid = bins[m] >= 0;
            int head, len;
            wave_runs(bins[m], valid, lane, head, len);
            if (valid && head == lane && bins[m] - w0 < SORT_WIN) atomicAdd(&cnt[bins[m] - w0], len);
        }
        __syncthreads();
        // reserve each bin's range for this chunk: one global atomic per bin
        for (int q = threadIdx.x; q < SORT_WIN; q += 256) {
            const int c = cnt[q];
            if (c) cnt[q] = atomicAdd(&off[w0 + q], c);
            rk[q] = 0;
        }
        __syncthreads();
        // rank within the bin (LDS), then move
        int dix[SORT_PER_THREAD];                      // destination slot, -1 if none
#pragma unroll
        for (int m = 0; m < SORT_PER_THREAD; ++m) {
            const int bin = bins[m];
            const bool valid = bin >= 0;
            int head, len;
            wave_runs(bin, valid, lane, head, len);
            int first = 0;
            if (valid && head == lane) {
                const int w = bin - w0;
                if (w < SORT_WIN) first = cnt[w] + atomicAdd(&rk[w], len);
                else first = atomicAdd(&off[bin], len);
            }
            first = __shfl(first, head, 64);
            dix[m] = valid ? first + (lane - head) : -1;
        }
        if constexpr (sizeof(T) == 4) {
            // FP32: the position words are already held; the velocities and
            // ids move in groups of four slots, every load of a group issued
            // before its stores (one memory round trip per group)
            const float *__restrict__ svr = (const float *)src.vr;
            const float *__restrict__ svt = (const float *)src.vt;
            const float *__restrict__ svz = (const float *)src.vz;
            const uint32_t *__restrict__ sid = src.id;
            uint32_t *__restrict__ dfr = (uint32_t *)dst.fr;
            uint32_t *__restrict__ dfz = (uint32_t *)dst.fz;
            float *__restrict__ dvr = (float *)dst.vr;
            float *__restrict__ dvt = (float *)dst.vt;
            float *__restrict__ dvz = (float *)dst.vz;
            uint32_t *__restrict__ did = dst.id;
#pragma unroll
            for (int g = 0; g < SORT_PER_THREAD; g += 4) {
                float a[4], b[4], c[4];
                uint32_t e[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t p = base + (g + u) * 256 + threadIdx.x;
                    const int64_t pl = dix[g + u] >= 0 ? p : 0;   // slot 0: a valid address
                    a[u] = svr[pl];
                    b[u] = svt[pl];
                    c[u] = svz[pl];
                    e[u] = sid[pl];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int d = dix[g + u];
                    if (d >= 0) {
                        dfr[d] = wr[g + u];
                        dfz[d] = wz[g + u];
                        dvr[d] = a[u];
                        dvt[d] = b[u];
                        dvz[d] = c[u];
                        did[d] = e[u];
                    }
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < SORT_PER_THREAD; ++m)
                if (dix[m] >= 0) copy_slot(src, dst, base + m * 256 + threadIdx.x, (int64_t)dix[m]);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < SORT_WIN; q += 256) cnt[q] = 0;
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_sort_scatter(SpeciesDev<T> src, SpeciesDev<T> dst,
                                                       const DevScalars *sc, int species,
                                                       int32_t nr, int32_t *off)
{
    sort_scatter_body(src, dst, sc, species, nr, off, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void k_sort_finish(DevScalars *sc, int species)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->count[species] = sc->sort_total[species];
}

// ---- batched forms: the sort of one species in every run of a batch, one
// launch per kernel; a block finds its run from the block offsets
template <typename T>
__device__ __forceinline__ int sort_run(const SortBatch<T> &B, int b)
{
    int lo = 0, hi = B.nruns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(256) k_sort_zero_b(SortBatch<T> B)
{
    const int b = (int)blockIdx.x, r = sort_run(B, b);
    const SortJob<T> &J = B.job[r][B.species];
    const int nb = B.off[r + 1] - B.off[r];
    for (int q = (b - B.off[r]) * 256 + threadIdx.x; q < J.nbins; q += nb * 256) J.hist[q] = 0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_sort_hist_b(SortBatch<T> B)
{
    const int b = (int)blockIdx.x, r = sort_run(B, b);
    const SortJob<T> &J = B.job[r][B.species];
    sort_hist_body(J.src, J.sc, B.species, J.nr, J.hist, b - B.off[r], B.off[r + 1] - B.off[r]);
}

template <typename T>
__global__ void k_scan_tiles_b(SortBatch<T> B)
{
    const int b = (int)blockIdx.x, r = sort_run(B, b);
    const SortJob<T> &J = B.job[r][B.species];
    scan_tiles_body(J.hist, J.nbins, J.block_sums, b - B.off[r]);
}

// one block per run
template <typename T>
__global__ void __launch_bounds__(1024) k_scan_top_b(SortBatch<T> B)
{
    const SortJob<T> &J = B.job[blockIdx.x][B.species];
    scan_top_body(J.block_sums, (J.nbins + SCAN_TILE - 1) / SCAN_TILE, J.sc, B.species);
}

template <typename T>
__global__ void __launch_bounds__(SCAN_TILE) k_scan_down_b(SortBatch<T> B)
{
    const int b = (int)blockIdx.x, r = sort_run(B, b);
    const SortJob<T> &J = B.job[r][B.species];
    scan_down_body(J.hist, J.nbins, J.block_sums, b - B.off[r]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_sort_scatter_b(SortBatch<T> B)
{
    const int b = (int)blockIdx.x, r = sort_run(B, b);
    const SortJob<T> &J = B.job[r][B.species];
    sort_scatter_body(J.src, J.dst, J.sc, B.species, J.nr, J.hist, b - B.off[r],
                      B.off[r + 1] - B.off[r]);
}

// one thread per run
template <typename T>
__global__ void k_sort_finish_b(SortBatch<T> B)
{
    const int r = (int)threadIdx.x;
    if (r >= B.nruns) return;
    DevScalars *sc = B.job[r][B.species].sc;
    sc->count[B.species] = sc->sort_total[B.species];
}

}  // namespace

int sort_blocks(int64_t cap)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (cap + SORT_CHUNK - 1) / SORT_CHUNK));
}

template <typename T>
void launch_sort_b(SortBatch<T> B, const int64_t *cap, hipStream_t s)
{
    const int n = B.nruns;
    auto offsets = [&](auto blocks_of) {
        B.off[0] = 0;
        for (int r = 0; r < n; ++r) B.off[r + 1] = B.off[r] + blocks_of(r);
        return B.off[n];
    };
    auto ntiles = [&](int r) { return (B.nbins[r] + SCAN_TILE - 1) / SCAN_TILE; };
    int g = offsets([&](int r) { return std::max(1, std::min(256, (B.nbins[r] + 255) / 256)); });
    hipLaunchKernelGGL((k_sort_zero_b<T>), dim3(g), dim3(256), 0, s, B);
    g = offsets([&](int r) { return sort_blocks(cap[r]); });
    hipLaunchKernelGGL((k_sort_hist_b<T>), dim3(g), dim3(256), 0, s, B);
    const SortBatch<T> Bh = B;
    g = offsets(ntiles);
    hipLaunchKernelGGL((k_scan_tiles_b<T>), dim3(g), dim3(256), 0, s, B);
    hipLaunchKernelGGL((k_scan_top_b<T>), dim3(n), dim3(1024), 0, s, B);
    hipLaunchKernelGGL((k_scan_down_b<T>), dim3(g), dim3(SCAN_TILE), 0, s, B);
    hipLaunchKernelGGL((k_sort_scatter_b<T>), dim3(Bh.off[n]), dim3(256), 0, s, Bh);
    hipLaunchKernelGGL((k_sort_finish_b<T>), dim3(1), dim3(MAX_BATCH), 0, s, B);
}

template <typename T>
void launch_sort(SpeciesDev<T> src, SpeciesDev<T> dst, DevScalars *sc, int species,
                 int32_t *hist, int32_t *block_sums, int32_t nr, int32_t nz, int64_t cap,
                 hipStream_t s)
{
    const int32_t nbins = nr * nz;
    const int ntiles = (nbins + SCAN_TILE - 1) / SCAN_TILE;
    launch_zero(hist, (int64_t)nbins * 4, s);
    const int blocks = sort_blocks(cap);
    hipLaunchKernelGGL((k_sort_hist<T>), dim3(blocks), dim3(256), 0, s, src, sc, species, nr, hist);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, hist, nbins, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, block_sums, ntiles, sc, species);
    hipLaunchKernelGGL(k_scan_down, dim3(ntiles), dim3(SCAN_TILE), 0, s, hist, nbins, block_sums);
    hipLaunchKernelGGL((k_sort_scatter<T>), dim3(blocks), dim3(256), 0, s, src, dst, sc, species,
                       nr, hist);
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(64), 0, s, sc, species);
}

template void launch_sort<float>(SpeciesDev<float>, SpeciesDev<float>, DevScalars *, int,
                                 int32_t *, int32_t *, int32_t, int32_t, int64_t, hipStream_t);
template void launch_sort<double>(SpeciesDev<double>, SpeciesDev<double>, DevScalars *, int,
                                  int32_t *, int32_t *, int32_t, int32_t, int64_t, hipStream_t);
template void launch_sort_b<float>(SortBatch<float>, const int64_t *, hipStream_t);
template void launch_sort_b<double>(SortBatch<double>, const int64_t *, hipStream_t);

}  // namespace pic
