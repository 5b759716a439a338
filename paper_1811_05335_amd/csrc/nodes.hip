// Node preprocessing: wrap onto the torus, stencil base and offset per dimension, counting sort
// of the nodes by grid cell (tile-major keys), and the CSR over cells from which both the
// spreading tiles and the grid-index -> node lists I(l) of (3.29) are read.
#include "internal.hpp"

#include <algorithm>

#include <limits.h>

namespace infft {

__global__ void k_fill_i32(int* p, int64_t n, int v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// exclusive scan over cells: blocks of SCAN_BLOCK cells, SCAN_T threads x SCAN_ITEMS each
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_BLOCK = SCAN_T * SCAN_ITEMS;
// Up to this many scan blocks the node sort adds the block offsets inside the scatter and the
// cell sort (each workgroup scans the block totals itself) instead of a launch of its own.
constexpr int SCAT_MAXB = 4096;

// Exclusive prefix sums of v[0..n) (n <= SCAT_MAXB) into s_out[0..n), by a workgroup of 256
// threads, 256 values at a time.
__device__ inline void block_prefix_small(const int* __restrict__ v, int n, int* s_out, int* s_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int carry = 0;
    for (int b0 = 0; b0 < n; b0 += 256) {
        const int i = b0 + (int)threadIdx.x;
        const int x = i < n ? v[i] : 0;
        int inc = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        int run = inc - x + carry;
        for (int w = 0; w < wave; ++w) run += s_w[w];
        if (i < n) s_out[i] = run;
        carry += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

static int grid_for(int64_t n, int threads, int cap = 65536) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

void launch_fill_i32(int* p, int64_t n, int v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
}

void launch_fill_bytes0(void* p, int64_t nbytes, hipStream_t s) {
    if (nbytes <= 0) return;
    // all workspace regions are 4-byte multiples
    const int64_t n = nbytes / 4;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, (uint32_t*)p, n);
}

__global__ void k_status_init(long long* st, int keep_node_words) {
    const int i = threadIdx.x;
    if (i >= STATUS_WORDS || (keep_node_words && i == ST_NONFINITE)) return;
    st[i] = (i == ST_MIN_N) ? LLONG_MAX : 0;
}

void launch_status_init(long long* status, int keep_node_words, hipStream_t s) {
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, status, keep_node_words);
}


// Start of the node preprocessing in one launch: the status block, the per-cell counters and fill
// cursors, and the four list counters.
__global__ void k_nodes_reset(long long* st, int* counts, int64_t ncounts, int* fill, int64_t nfill, int* lcount) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < ncounts) counts[i] = 0;
    if (i < nfill) fill[i] = 0;
    if (i < 8) lcount[i] = 0;   // list counters and the tickets of the tiers that clear them
    if (i < STATUS_WORDS) st[i] = (i == ST_MIN_N) ? LLONG_MAX : 0;
}

void launch_nodes_reset(long long* status, int* counts, int64_t ncounts, int* fill, int64_t nfill, int* lcount,
                        hipStream_t s) {
    const int64_t n = std::max<int64_t>(std::max<int64_t>(ncounts, nfill), STATUS_WORDS);
    hipLaunchKernelGGL(k_nodes_reset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, status, counts, ncounts,
                       fill, nfill, lcount);
}

// Per node: wrap, t = x M_sigma, l0 = ceil(t - m), u = t - l0.  The float64 operations are
// kept separate (no contraction into fused multiply-adds) so the stencil, and therefore the
// sparsity pattern of B and B_opt, follows exactly these roundings.
template <int D>
__device__ inline void prep_node(const Geo& g, const double* __restrict__ x, NodesDev& nd, int* __restrict__ counts,
                                 int64_t j, bool& bad) {
#pragma clang fp contract(off)
    int c[2] = {0, 0};
#pragma unroll
    for (int t = 0; t < D; ++t) {
        double xv = x[j * D + t];
        if (!isfinite(xv)) {
            bad = true;
            xv = 0.0;
        }
        const double xw = xv - floor(xv + 0.5);
        const double tt = xw * (double)g.Ms[t];
        const double l0 = ceil(tt - (double)g.m);
        const double u = tt - l0;
        int lm = (int)l0 % g.Ms[t];
        if (lm < 0) lm += g.Ms[t];
        ((double*)nd.xw)[j * D + t] = xw;
        nd.l0c[j * D + t] = lm;
        nd.uc[j * D + t] = u;
        c[t] = lm;
    }
    const int key = (int)cell_key(g, c[0], c[1]);
    nd.key[j] = key;
    atomicAdd(&counts[key], 1);
}

template <int D>
__global__ void __launch_bounds__(256) k_prep(Geo g, const double* __restrict__ x, NodesDev nd,
                                              int* __restrict__ counts, int* __restrict__ nonfinite) {
#pragma clang fp contract(off)
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool bad = false;
    if (j < g.N) prep_node<D>(g, x, nd, counts, j, bad);
    // the workgroup's count of non-finite nodes (the cell sort folds them into the status block)
    const int nbad = __syncthreads_count(bad);
    if (threadIdx.x == 0) nonfinite[blockIdx.x] = nbad;
}

int prep_blocks(const Geo& g) { return (int)((g.N + 255) / 256); }

void launch_prep_nodes(const Geo& g, const double* x, NodesDev nd, int* counts, int* nonfinite, hipStream_t s) {
    const int blocks = prep_blocks(g);
    if (g.d == 1)
        hipLaunchKernelGGL(k_prep<1>, dim3(blocks), dim3(256), 0, s, g, x, nd, counts, nonfinite);
    else
        hipLaunchKernelGGL(k_prep<2>, dim3(blocks), dim3(256), 0, s, g, x, nd, counts, nonfinite);
}

// local/bsum (bsum non-null): the cell starts are the in-block exclusive sums `local` plus the
// sum of the preceding blocks' totals, which each workgroup scans itself; else nd.start holds them.
template <int D>
__global__ void __launch_bounds__(256) k_scatter(Geo g, NodesDev nd, const int* __restrict__ local,
                                                 const int* __restrict__ bsum, int nb, int* __restrict__ fill) {
    __shared__ int s_off[SCAT_MAXB + 1];
    __shared__ int s_w[4];
    if (bsum) block_prefix_small(bsum, nb, s_off, s_w);
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= g.N) return;
    const int key = nd.key[j];
    const int base = bsum ? local[key] + s_off[key / SCAN_BLOCK] : nd.start[key];
    const int pos = base + atomicAdd(&fill[key], 1);
    nd.perm[pos] = (int)j;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        nd.l0s[(int64_t)pos * D + t] = nd.l0c[j * D + t];
        nd.us[(int64_t)pos * D + t] = nd.uc[j * D + t];
    }
}



// ------------------------------------------------------------------ deterministic order in a cell
// The scatter places the nodes of one cell in atomic order.  Sorting each cell's range by caller
// index makes the sorted order, and with it every member order of the local problems, a function
// of the input alone.  Cells of up to CELL_SORT_SMALL nodes are sorted by one thread in place;
// larger cells (dense 2-D centres) by the workgroup that found them, with a bitonic sort in LDS.

constexpr int CELL_SORT_SMALL = 32;
constexpr int CELL_SORT_BIG = 4096;

template <int D>
__device__ inline void refresh_sorted(NodesDev& nd, int pos) {
    const int j = nd.perm[pos];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        nd.l0s[(int64_t)pos * D + t] = nd.l0c[(int64_t)j * D + t];
        nd.us[(int64_t)pos * D + t] = nd.uc[(int64_t)j * D + t];
    }
}

// One workgroup per CELL_SORT_TPB cells: each thread sorts a small cell by itself; the cells above
// CELL_SORT_SMALL nodes are collected in LDS and sorted afterwards by the whole workgroup.
// The last kernel of the node preprocessing also ends it: each thread clears its cell's counter
// and fill cursor (read for the last time by the scan and the scatter), so the next call starts
// from zeros without a reset launch, and workgroup 0 writes the status block: the node words
// (the non-finite count, summed from the preprocessing's per-workgroup counts) and the solve
// words at their initial values.
constexpr int CELL_SORT_TPB = 256;

// bsum non-null: counts holds the in-block exclusive sums of the cell counts and fill the counts
// (the scatter's cursors); the workgroup adds its scan block's offset and writes nd.start.
template <int D>
__global__ void __launch_bounds__(CELL_SORT_TPB) k_cell_sort(Geo g, NodesDev nd, int* __restrict__ counts,
                                                             int* __restrict__ fill, const int* __restrict__ bsum,
                                                             const int* __restrict__ nonfinite, int nprep,
                                                             long long* __restrict__ status) {
    __shared__ int buf[CELL_SORT_BIG];
    __shared__ int s_big[CELL_SORT_TPB];
    __shared__ int s_bigse[CELL_SORT_TPB][2];
    __shared__ int s_nbig;
    __shared__ int s_off;
    __shared__ long long s_bad;
    if (threadIdx.x == 0) {
        s_nbig = 0;
        s_bad = 0;
    }
    if (bsum && threadIdx.x < 64) {
        // the cells of a workgroup lie in one scan block (SCAN_BLOCK is a multiple of the TPB)
        const int64_t b = (blockIdx.x * (int64_t)CELL_SORT_TPB) / SCAN_BLOCK;
        int acc = 0;
        for (int64_t i = threadIdx.x; i < b; i += 64) acc += bsum[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (threadIdx.x == 0) s_off = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        long long bad = 0;
        for (int b = threadIdx.x; b < nprep; b += blockDim.x) bad += nonfinite[b];
        if (bad) atomicAdd((unsigned long long*)&s_bad, (unsigned long long)bad);
    }
    const int64_t c = blockIdx.x * (int64_t)CELL_SORT_TPB + threadIdx.x;
    if (c < g.G) {
        int s, e;
        if (bsum) {
            s = counts[c] + s_off;
            e = s + fill[c];
            nd.start[c] = s;
            if (c == g.G - 1) nd.start[g.G] = e;
        } else {
            s = nd.start[c];
            e = nd.start[c + 1];
        }
        counts[c] = 0;
        fill[c] = 0;
        const int cnt = e - s;
        if (cnt > CELL_SORT_SMALL) {
            const int k = atomicAdd(&s_nbig, 1);
            s_big[k] = (int)c;
            s_bigse[k][0] = s;
            s_bigse[k][1] = e;
        } else if (cnt > 1) {
            for (int i = s + 1; i < e; ++i) {  // insertion sort of perm[s..e)
                const int v = nd.perm[i];
                int k = i - 1;
                while (k >= s && nd.perm[k] > v) {
                    nd.perm[k + 1] = nd.perm[k];
                    --k;
                }
                nd.perm[k + 1] = v;
            }
            for (int i = s; i < e; ++i) refresh_sorted<D>(nd, i);
        }
    }
    __syncthreads();
    const int nbig = s_nbig;
    for (int b = 0; b < nbig; ++b) {
        const int s = s_bigse[b][0], e = s_bigse[b][1];
        const int cnt = e - s;
        if (cnt > CELL_SORT_BIG) continue;  // left in scatter order
        int n2 = 1;
        while (n2 < cnt) n2 <<= 1;
        for (int i = threadIdx.x; i < n2; i += blockDim.x) buf[i] = (i < cnt) ? nd.perm[s + i] : INT_MAX;
        __syncthreads();
        for (int k = 2; k <= n2; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const int a = buf[i], bb = buf[ixj];
                        const bool up = (i & k) == 0;
                        if ((a > bb) == up) {
                            buf[i] = bb;
                            buf[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) nd.perm[s + i] = buf[i];
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) refresh_sorted<D>(nd, s + i);
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x < STATUS_WORDS) {
        const int i = threadIdx.x;
        status[i] = (i == ST_NONFINITE) ? s_bad : (i == ST_MIN_N) ? LLONG_MAX : 0;
    }
}



// ------------------------------------------------------------------ exclusive scan
// Three passes: per-block scan (256 threads x 8 items), scan of the block totals in one block,
// then the block offsets are added.  out has n+1 entries (out[n] = total).


__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
    // inclusive scan inside each wave, then across the 4 wave totals
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_T / 64; ++w) {
        const int s = sh[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// in and out may be the same array (each thread reads its items before writing them).
__global__ void k_scan1(const int* in, int* out, int64_t n, int* bsum) {
    __shared__ int sh[SCAN_T / 64];
    const int64_t base = blockIdx.x * (int64_t)SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int total;
    int run = block_exclusive_scan(s, sh, &total);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Adds the sum of the preceding blocks' totals.  A workgroup of 256 lies inside one scan block, so
// its first wavefront sums those totals itself (at most 2048 of them) instead of a separate scan.
__global__ void k_scan3(int* __restrict__ out, int64_t n, const int* __restrict__ bsum, int64_t nb) {
    __shared__ int s_off;
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x;
    const int64_t b = i0 / SCAN_BLOCK;                       // scan block of this workgroup
    if (threadIdx.x < 64) {
        int acc = 0;
        for (int64_t j = threadIdx.x; j < b; j += 64) acc += bsum[j];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (threadIdx.x == 0) s_off = acc;
    }
    __syncthreads();
    const int64_t i = i0 + threadIdx.x;
    if (i < n) out[i] += s_off;
    if (i == n) out[n] = s_off + (b < nb ? bsum[b] : 0);   // the grand total
}

int64_t scan_blocksum_len(int64_t n) { return (n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1; }

void launch_exclusive_scan(const int* in, int* out, int64_t n, int* blocksums, hipStream_t s) {
    const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    hipLaunchKernelGGL(k_scan1, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, blocksums);
    hipLaunchKernelGGL(k_scan3, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, out, n,
                       (const int*)blocksums, nb);
}

// ------------------------------------------------------------------ the node sort
// Counting sort of the nodes by cell from the per-cell counts of k_prep: the scan of the counts,
// the scatter, and the sort inside each cell (which also writes nd.start and leaves counts and fill
// cursors at zero).  Up to SCAT_MAXB scan blocks the block offsets are added inside the scatter
// and the cell sort (three launches), else by a scan pass of their own (four).
static_assert(SCAN_BLOCK % CELL_SORT_TPB == 0, "a cell-sort workgroup lies in one scan block");

void launch_sort_nodes(const Geo& g, NodesDev nd, int* counts, int* fill, int* bsum, const int* nonfinite,
                       long long* status, hipStream_t s) {
    const int64_t nb = (g.G + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const bool fused = nb <= SCAT_MAXB;
    const int* bs = nullptr;
    if (fused) {
        // in-block exclusive sums in place of the counts
        hipLaunchKernelGGL(k_scan1, dim3((unsigned)nb), dim3(SCAN_T), 0, s, (const int*)counts, counts, g.G, bsum);
        bs = bsum;
    } else {
        launch_exclusive_scan(counts, nd.start, g.G, bsum, s);
    }
    const int* local = fused ? counts : nullptr;
    const int sblocks = (int)((g.N + 255) / 256);
    if (g.d == 1)
        hipLaunchKernelGGL(k_scatter<1>, dim3(sblocks), dim3(256), 0, s, g, nd, local, bs, (int)nb, fill);
    else
        hipLaunchKernelGGL(k_scatter<2>, dim3(sblocks), dim3(256), 0, s, g, nd, local, bs, (int)nb, fill);
    const unsigned cblocks = (unsigned)((g.G + CELL_SORT_TPB - 1) / CELL_SORT_TPB);
    const int np = prep_blocks(g);
    if (g.d == 1)
        hipLaunchKernelGGL(k_cell_sort<1>, dim3(cblocks), dim3(CELL_SORT_TPB), 0, s, g, nd, counts, fill, bs,
                           nonfinite, np, status);
    else
        hipLaunchKernelGGL(k_cell_sort<2>, dim3(cblocks), dim3(CELL_SORT_TPB), 0, s, g, nd, counts, fill, bs,
                           nonfinite, np, status);
}

// ------------------------------------------------------------------ B_opt export

__global__ void k_export_B(int64_t N, int T, const int* __restrict__ perm, const double2* __restrict__ B,
                           double2* __restrict__ rows) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N * T) return;
    const int64_t tau = i / N, p = i - tau * N;
    rows[(int64_t)perm[p] * T + tau] = B[i];
}

void launch_export_B(const Geo& g, const int* perm, const double2* B, double2* rows, hipStream_t s) {
    int T = 2 * g.m + 1;
    if (g.d == 2) T *= T;
    const int64_t n = g.N * T;
    hipLaunchKernelGGL(k_export_B, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.N, T, perm, B,
                       rows);
}

}  // namespace infft
