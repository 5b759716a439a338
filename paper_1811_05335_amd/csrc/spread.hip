// The sparse factor B of the NFFT (2.6) and its optimised replacement B_opt (Algorithm 3.17):
//   interp     f_j = sum_tau g[l0_j + tau] w~_m(x_j - l/M_sigma)           (last step of A ~ BFD)
//   spread     g~_l = sum_j f_j w~_m(x_j - l/M_sigma)  or  sum_j conj(B_opt[j,l]) f_j
//              (first step of the adjoint (2.8) and of the modified adjoint (3.32))
//   interp_B   f_j = sum_tau B_opt[j, tau] g[l0_j + tau]                    (B_opt F D, Remark 3.24)
//   grad_x     d/dx_j of the interpolation through the window derivative
//
// The Kaiser-Bessel window w(v) = sinh(b sqrt(m^2 - v^2)) / (pi sqrt(m^2 - v^2)) is evaluated in
// registers from per-tap polynomials fitted at plan time (w is an entire function of v, so each
// unit interval needs degree 10 in FP32 and 16 in FP64); whether a tap lies in the closed support
// |v| <= m is decided in float64 from the stored offsets for both precisions.
//
// Spreading runs one workgroup per grid tile (TS0 x TS1 cells).  The nodes of a tile are a
// contiguous range of the sorted node order; their contributions are accumulated with LDS
// atomics into the tile plus a 2m-wide halo on the + side of each dimension.  The tile interior
// is then written with plain stores and the halo strips to separate buffers, which the first
// pass of the following FFT adds in (no global atomics, no zero-fill of the grid).
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace infft {

// Window values of the 2m+1 taps of one node.  Taps tau < 2m: Horner in y of the plan's polynomial
// of that tap (membership |u - tau| <= m still decided in float64); tap 2m reaches the window only
// when u - 2m rounds to -m (u at m), where the window equals its edge value b/pi.
template <typename R, int W>
__device__ inline void window_row(const Geo& g, double u, R* w) {
    constexpr int NC = WPoly<R>::NC;
    const R* cf = (const R*)g.wpoly;
    const R y = (R)(2.0 * (u - (double)(g.m - 1)) - 1.0);
    if constexpr ((W - 1) * NC > 135) {
        // many coefficients (FP64 from m = 4, FP32 from m = 7): the same Horner steps per tap with
        // the power loop outermost and rolled, so that one coefficient per tap is live.  Unrolled,
        // a kernel that evaluates rows in a loop keeps every coefficient in vector registers
        // (the FP64 1-D spreading at m = 6 held 452 of them and ran one wave per SIMD)
#pragma unroll
        for (int tau = 0; tau < W - 1; ++tau) w[tau] = cf[tau * NC + NC - 1];
#pragma unroll 1
        for (int k = NC - 2; k >= 0; --k) {
#pragma unroll
            for (int tau = 0; tau < W - 1; ++tau) w[tau] = w[tau] * y + cf[tau * NC + k];
        }
#pragma unroll
        for (int tau = 0; tau < W - 1; ++tau) w[tau] = (fabs(u - (double)tau) <= (double)g.m) ? w[tau] : (R)0;
    } else {
#pragma unroll
        for (int tau = 0; tau < W - 1; ++tau) {
            R acc = cf[tau * NC + NC - 1];
#pragma unroll
            for (int k = NC - 2; k >= 0; --k) acc = acc * y + cf[tau * NC + k];
            w[tau] = (fabs(u - (double)tau) <= (double)g.m) ? acc : (R)0;
        }
    }
    w[W - 1] = edge_tap_member(u, g.m) ? (R)(g.b / M_PI) : (R)0;
}

// Derivatives d w / d v of the same taps (times `scale`): d/dv = 2 d/dy; at the on-grid edge tap
// the one-sided derivative inside the support, m b^3 / (3 pi).
template <typename R, int W>
__device__ inline void window_deriv_row(const Geo& g, double u, R scale, R* dw) {
    constexpr int NC = WPoly<R>::NC;
    const R* cf = (const R*)g.wpoly;
    const R y = (R)(2.0 * (u - (double)(g.m - 1)) - 1.0);
#pragma unroll
    for (int tau = 0; tau < W - 1; ++tau) {
        R p = cf[tau * NC + NC - 1], dp = (R)0;
#pragma unroll
        for (int k = NC - 2; k >= 0; --k) {
            dp = dp * y + p;
            p = p * y + cf[tau * NC + k];
        }
        dw[tau] = (fabs(u - (double)tau) <= (double)g.m) ? (R)2 * scale * dp : (R)0;
    }
    dw[W - 1] = edge_tap_member(u, g.m) ? (R)(scale * (double)g.m * g.b * g.b * g.b / (3.0 * M_PI)) : (R)0;
}

// One tap with a tap index known only at run time (gather over the nodes reaching one cell).
template <typename R>
__device__ inline R window_tap(const Geo& g, double u, int tau) {
    constexpr int NC = WPoly<R>::NC;
    if (tau >= 2 * g.m) return edge_tap_member(u, g.m) ? (R)(g.b / M_PI) : (R)0;
    if (fabs(u - (double)tau) > (double)g.m) return (R)0;
    const R* cf = (const R*)g.wpoly + tau * NC;
    const R y = (R)(2.0 * (u - (double)(g.m - 1)) - 1.0);
    R acc = cf[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) acc = acc * y + cf[k];
    return acc;
}

__device__ inline int wrap_add(int a, int t, int Ms) {
    const int v = a + t;
    return v >= Ms ? v - Ms : v;
}

// ------------------------------------------------------------------ interpolation (trafo)

template <typename R, int D, int W>
__device__ inline void interp_item(const Geo& g, const NodesDev& nd, const cx<R>* __restrict__ grid, int64_t grs,
                                   cx<R>* __restrict__ f, int nrhs, int64_t j) {
    using C = cx<R>;
    if (j >= g.N) return;
    const R b = (R)g.b;
    R w0[W], w1[W];
    window_row<R, W>(g, nd.uc[j * D], w0);
    const int a0 = nd.l0c[j * D];
    int a1 = 0;
    if (D == 2) {
        window_row<R, W>(g, nd.uc[j * D + 1], w1);
        a1 = nd.l0c[j * D + 1];
    }
    for (int r = 0; r < nrhs; ++r) {
        const C* gr = grid + r * grs;
        C acc = cmake((R)0, (R)0);
        if (D == 1) {
#pragma unroll
            for (int t = 0; t < W; ++t) {
                const C v = gr[wrap_add(a0, t, g.Ms[0])];
                acc.x += w0[t] * v.x;
                acc.y += w0[t] * v.y;
            }
        } else {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                const C* row = gr + (int64_t)wrap_add(a0, t0, g.Ms[0]) * g.Ms[1];
                C s = cmake((R)0, (R)0);
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const C v = row[wrap_add(a1, t1, g.Ms[1])];
                    s.x += w1[t1] * v.x;
                    s.y += w1[t1] * v.y;
                }
                acc.x += w0[t0] * s.x;
                acc.y += w0[t0] * s.y;
            }
        }
        f[r * g.N + j] = acc;
    }
}

template <typename R, int D, int W>
__global__ void __launch_bounds__(256) k_interp(Geo g, NodesDev nd, const cx<R>* __restrict__ grid,
                                                int64_t grs, cx<R>* __restrict__ f, int nrhs) {
    interp_item<R, D, W>(g, nd, grid, grs, f, nrhs, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------------ interpolation with B_opt

template <typename R, int D, int W>
__device__ inline void interp_B_item(const Geo& g, const NodesDev& nd, const cx<R>* __restrict__ grid, int64_t grs,
                                     const cx<R>* __restrict__ B, cx<R>* __restrict__ f, int nrhs, int64_t p) {
    using C = cx<R>;
    if (p >= g.N) return;
    const int j = nd.perm[p];
    const int a0 = nd.l0s[p * D];
    const int a1 = (D == 2) ? nd.l0s[p * D + 1] : 0;
    // 2-D with many taps: the outer tap loop stays rolled so the loads of one row are in flight at a
    // time (unrolled, all W^2 entries of B and the grid would be hoisted and spill)
    constexpr int UNR0 = (D == 2 && W * W * (int)sizeof(C) > 1024) ? 1 : W;
    for (int r = 0; r < nrhs; ++r) {
        const C* gr = grid + r * grs;
        C acc = cmake((R)0, (R)0);
#pragma unroll UNR0
        for (int t0 = 0; t0 < W; ++t0) {
            if (D == 1) {
                const C wv = B[(int64_t)t0 * g.N + p];
                const C v = gr[wrap_add(a0, t0, g.Ms[0])];
                acc = cadd(acc, cmul(wv, v));
            } else {
                const C* row = gr + (int64_t)wrap_add(a0, t0, g.Ms[0]) * g.Ms[1];
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const C wv = B[(int64_t)(t0 * W + t1) * g.N + p];
                    acc = cadd(acc, cmul(wv, row[wrap_add(a1, t1, g.Ms[1])]));
                }
            }
        }
        f[r * g.N + j] = acc;
    }
}

template <typename R, int D, int W>
__global__ void __launch_bounds__(256) k_interp_B(Geo g, NodesDev nd, const cx<R>* __restrict__ grid,
                                                  int64_t grs, const cx<R>* __restrict__ B,
                                                  cx<R>* __restrict__ f, int nrhs) {
    interp_B_item<R, D, W>(g, nd, grid, grs, B, f, nrhs, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------------ tiled spreading

template <typename R> __device__ inline void lds_add(R* p, R v) { atomicAdd(p, v); }

template <typename T> __device__ inline void gadd(T* p, T v) { unsafeAtomicAdd(p, v); }

template <typename R, int D, int W, bool USEB>
__global__ void __launch_bounds__(256) k_spread(Geo g, NodesDev nd, const cx<R>* __restrict__ f,
                                                const cx<R>* __restrict__ B, cx<R>* __restrict__ grid,
                                                int64_t grs, cx<R>* __restrict__ h0, cx<R>* __restrict__ h1,
                                                cx<R>* __restrict__ h01, int64_t hrs0, int64_t hrs1,
                                                int64_t hrs01, int nrhs, int rchunk, SpreadWork wk) {
    using C = cx<R>;
    extern __shared__ char smem_raw[];
    // [rc][E0][E1][2] in float64 for both precisions: LDS float32 atomic adds stall the issue of
    // LDS instructions many times longer than float64 ones here (measured), and the sums gain
    // accuracy besides
    double* acc = (double*)smem_raw;
    const int w2 = 2 * g.m;
    if ((int)blockIdx.x >= *wk.total) return;
    const int2 item = wk.items[blockIdx.x];
    const int tile = item.x;
    const int nch = wk.nchunk[tile];   // chunks of the tile: more than one -> atomic flush
    const int t0 = (D == 2) ? tile / g.ntile[1] : tile;
    const int t1 = (D == 2) ? tile - t0 * g.ntile[1] : 0;
    const int TS0 = g.TS[0], TS1 = (D == 2) ? g.TS[1] : 1;
    const int E0 = TS0 + w2, E1 = (D == 2) ? TS1 + w2 : 1;
    const int cells = E0 * E1;
    const int base0 = t0 * TS0, base1 = t1 * TS1;
    const int64_t kbeg = (int64_t)tile * TS0 * TS1;
    const int tbeg = nd.start[kbeg], tend = nd.start[kbeg + (int64_t)TS0 * TS1];
    const int pbeg = min(tbeg + item.y * wk.chunk, tend), pend = min(pbeg + wk.chunk, tend);
    const R b = (R)g.b;

    // blockIdx.y picks the chunk of right-hand sides: each workgroup holds rc of them in LDS
    {
        const int r0 = (int)blockIdx.y * rchunk;
        const int rc = min(rchunk, nrhs - r0);
        for (int c = threadIdx.x; c < 2 * rc * cells; c += blockDim.x) acc[c] = 0.0;
        __syncthreads();
        // Nodes are sorted by cell, so the lanes of a wave holding nodes of one cell form
        // contiguous segments whose taps hit the same LDS words.  When a wave has few segments
        // (a dense spot: hundreds of nodes per cell) each tap's contributions are first summed
        // along the segment with shuffles and only the segment's first lane adds them to LDS;
        // otherwise every lane adds its own.
        const int lane = threadIdx.x & 63;
        for (int base = pbeg; base < pend; base += blockDim.x) {
            const int p = base + threadIdx.x;
            const bool valid = p < pend;
            int j = 0, a0 = 0, a1 = 0;
            R w0[W], w1[W];
#pragma unroll
            for (int t = 0; t < W; ++t) w0[t] = w1[t] = (R)0;
            if (valid) {
                j = nd.perm[p];
                a0 = nd.l0s[(int64_t)p * D] - base0;
                a1 = (D == 2) ? nd.l0s[(int64_t)p * D + 1] - base1 : 0;
                if (!USEB) {
                    window_row<R, W>(g, nd.us[(int64_t)p * D], w0);
                    if (D == 2) window_row<R, W>(g, nd.us[(int64_t)p * D + 1], w1);
                }
            }
            const int cid = valid ? a0 * E1 + a1 : -1 - lane;
            const int prev = __shfl_up(cid, 1, 64);
            const bool head = lane == 0 || prev != cid;
            const uint64_t hm = __ballot(head);
            const bool reduce = __popcll(hm) <= 16;   // the same in every lane of the wave
            const uint64_t above = hm & ~((2ull << lane) - 1ull);
            const int seg_end = above ? __ffsll((unsigned long long)above) - 1 : 64;
            // B_opt entries: the W entries of tap row s0 + 1 are loaded while row s0 is added (rows
            // rolled, so one row is buffered; lanes past the chunk read a valid position, unused)
            const int64_t pb = valid ? p : pbeg;
            for (int rr = 0; rr < rc; ++rr) {
                const C fv = valid ? f[(int64_t)(r0 + rr) * g.N + j] : cmake((R)0, (R)0);
                double* a = acc + (int64_t)rr * cells * 2;
                C brow[USEB ? W : 1], bnext[USEB ? W : 1];
                if (USEB) {
#pragma unroll
                    for (int s1 = 0; s1 < W; ++s1) brow[s1] = B[(int64_t)s1 * g.N + pb];
                }
#pragma unroll(USEB ? 1 : W)
                for (int s0 = 0; s0 < W; ++s0) {
                    C fs;
                    if (!USEB) fs = cscale(fv, w0[s0]);
                    if (USEB) {
                        const int sn = min(s0 + 1, W - 1);
#pragma unroll
                        for (int s1 = 0; s1 < W; ++s1) bnext[s1] = B[(int64_t)(sn * W + s1) * g.N + pb];
                    }
#pragma unroll
                    for (int s1 = 0; s1 < W; ++s1) {
                        C v = cmake((R)0, (R)0);
                        if (USEB) {
                            if (valid) v = cmulc(fv, brow[s1]);
                        } else {
                            v = cscale(fs, w1[s1]);
                        }
                        const int cidx = (a0 + s0) * E1 + (a1 + s1);
                        if (reduce) {
#pragma unroll
                            for (int o = 1; o < 64; o <<= 1) {
                                const R x2 = __shfl_down(v.x, o, 64), y2 = __shfl_down(v.y, o, 64);
                                if (lane + o < seg_end) {
                                    v.x += x2;
                                    v.y += y2;
                                }
                            }
                            if (head && valid) {
                                lds_add(&a[2 * cidx], (double)v.x);
                                lds_add(&a[2 * cidx + 1], (double)v.y);
                            }
                        } else if (valid) {
                            lds_add(&a[2 * cidx], (double)v.x);
                            lds_add(&a[2 * cidx + 1], (double)v.y);
                        }
                    }
                    if (USEB) {
#pragma unroll
                        for (int s1 = 0; s1 < W; ++s1) brow[s1] = bnext[s1];
                    }
                }
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < rc * cells; c += blockDim.x) {
            const int rr = c / cells, cc = c - rr * cells;
            const int e0 = cc / E1, e1 = cc - e0 * E1;
            const C v = cmake((R)acc[2 * c], (R)acc[2 * c + 1]);
            const int64_t r = r0 + rr;
            C* dst;
            if (e0 < TS0 && e1 < TS1) {
                dst = &grid[r * grs + (int64_t)(base0 + e0) * g.Ms[1] + (base1 + e1)];
            } else if (e0 >= TS0 && e1 < TS1) {
                dst = &h0[r * hrs0 + ((int64_t)tile * w2 + (e0 - TS0)) * TS1 + e1];
            } else if (e0 < TS0) {
                dst = &h1[r * hrs1 + ((int64_t)tile * TS0 + e0) * w2 + (e1 - TS1)];
            } else {
                dst = &h01[r * hrs01 + ((int64_t)tile * w2 + (e0 - TS0)) * w2 + (e1 - TS1)];
            }
            if (nch == 1) {
                *dst = v;
            } else if (v.x != (R)0 || v.y != (R)0) {
                // a chunk's nodes reach a few rows of the tile; cells they miss hold exact zeros
                gadd(&dst->x, v.x);
                gadd(&dst->y, v.y);
            }
        }
        __syncthreads();
    }
}

// Work list of the tiled spreading: a tile with more nodes than one chunk (the dense centre of a
// polar or spiral trajectory) is split into chunks, each a workgroup, whose partial tiles are added
// with global atomics into the tile's (zeroed) cells and halo strips.
__global__ void k_spread_chunks(Geo g, NodesDev nd, int chunk, int* __restrict__ nchunk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntiles = g.ntile[0] * g.ntile[1];
    if (t >= ntiles) return;
    const int64_t per = (int64_t)g.TS[0] * g.TS[1];
    const int cnt = nd.start[(t + 1) * per] - nd.start[t * per];
    nchunk[t] = max(1, (cnt + chunk - 1) / chunk);
}

__global__ void k_spread_items(Geo g, const int* __restrict__ nchunk, const int* __restrict__ offs,
                               int2* __restrict__ items, int* __restrict__ total) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntiles = g.ntile[0] * g.ntile[1];
    if (t >= ntiles) return;
    for (int c = 0; c < nchunk[t]; ++c) items[offs[t] + c] = make_int2(t, c);
    if (t == ntiles - 1) *total = offs[t] + nchunk[t];
}

void launch_spread_worklist(const Geo& g, NodesDev nd, SpreadWork wk, int* offs, int* bsum, hipStream_t s) {
    const int ntiles = g.ntile[0] * g.ntile[1];
    const unsigned nb = (unsigned)((ntiles + 255) / 256);
    hipLaunchKernelGGL(k_spread_chunks, dim3(nb), dim3(256), 0, s, g, nd, wk.chunk, wk.nchunk);
    launch_exclusive_scan(wk.nchunk, offs, ntiles, bsum, s);
    hipLaunchKernelGGL(k_spread_items, dim3(nb), dim3(256), 0, s, g, (const int*)wk.nchunk, (const int*)offs,
                       wk.items, wk.total);
}

// Zeroes the cells and halo strips of split tiles for all right-hand sides.
template <typename R>
__global__ void __launch_bounds__(256) k_spread_zero_split(Geo g, SpreadWork wk, cx<R>* grid, int64_t grs,
                                                           cx<R>* h0, cx<R>* h1, cx<R>* h01, int64_t hrs0,
                                                           int64_t hrs1, int64_t hrs01, int nrhs) {
    const int tile = blockIdx.x;
    if (wk.nchunk[tile] == 1) return;
    const int w2 = 2 * g.m, TS0 = g.TS[0], TS1 = g.TS[1];
    const int t0 = tile / g.ntile[1], t1 = tile - t0 * g.ntile[1];
    const int E0 = TS0 + w2, E1 = TS1 + w2, cells = E0 * E1;
    const cx<R> z = cmake((R)0, (R)0);
    for (int c = threadIdx.x; c < nrhs * cells; c += blockDim.x) {
        const int r = c / cells, cc = c - r * cells;
        const int e0 = cc / E1, e1 = cc - e0 * E1;
        if (e0 < TS0 && e1 < TS1) grid[r * grs + (int64_t)(t0 * TS0 + e0) * g.Ms[1] + (t1 * TS1 + e1)] = z;
        else if (e0 >= TS0 && e1 < TS1) h0[r * hrs0 + ((int64_t)tile * w2 + (e0 - TS0)) * TS1 + e1] = z;
        else if (e0 < TS0) h1[r * hrs1 + ((int64_t)tile * TS0 + e0) * w2 + (e1 - TS1)] = z;
        else h01[r * hrs01 + ((int64_t)tile * w2 + (e0 - TS0)) * w2 + (e1 - TS1)] = z;
    }
}

// ------------------------------------------------------------------ 1-D spreading, tiled
// One workgroup per tile of TS consecutive cells.  The nodes reaching the tile (stencil base in
// c0-2m .. c0+TS-1, a contiguous range of the sorted order, two at the wrap) are staged in LDS in
// chunks: per node its 2m+1 weights (window taps or B_opt entries, the latter read coalesced
// from the [tap][node] layout) and its samples for RC right-hand sides (gathered from the
// caller's order, all loads of a chunk in flight together).  Then thread t sums for cell c0+t
// over the nodes of cells c0+t-2m .. c0+t, a contiguous range of the staged nodes.

constexpr int SP1_TS = 256;     // cells per tile (threads per workgroup)
// Staged nodes per chunk: 256, and for one right-hand side as many as about 40 KB of LDS holds (up
// to 512), so that a tile at about one node per cell (256 cells plus the 2m-cell halo) is staged
// in one chunk, with one latency chain of loads, instead of a full chunk and a short second one.
template <typename Wt, typename C, int W, int RC> constexpr int sp1_cap() {
    constexpr int per = W * (int)sizeof(Wt) + RC * (int)sizeof(C) + (int)sizeof(int);
    constexpr int c = 40960 / per / 64 * 64;
    return (RC > 1 || c < 256) ? 256 : (c > 512 ? 512 : c);
}

// Position of the first node of tile-relative cell `rel` in the tile's node sequence, and the
// sorted position of sequence index i.  lo = c0 - 2m may be negative (the window wraps).
struct Tile1 {
    int lo, Ms;
    int sA, nA, sB;   // segment A: cells Ms+lo .. Ms-1 (only when lo < 0); segment B from cell max(lo, 0)
    __device__ Tile1(const NodesDev& nd, int c0, int m2, int Ms_) : Ms(Ms_) {
        lo = c0 - m2;
        if (lo < 0) {
            sA = nd.start[Ms + lo];
            nA = nd.start[Ms] - sA;
            sB = nd.start[0];
        } else {
            sA = nA = 0;
            sB = nd.start[lo];
        }
    }
    __device__ int pos(const NodesDev& nd, int rel) const {
        if (lo < 0 && rel <= -lo) return nd.start[Ms + lo + rel] - sA;
        return nA + nd.start[lo + rel] - sB;
    }
    __device__ int sorted(int i) const { return i < nA ? sA + i : sB + (i - nA); }
};

template <typename R, int W, bool USEB, int RC>
__device__ inline void spread1d_tile(const Geo& g, const NodesDev& nd, const cx<R>* __restrict__ f,
                                     const cx<R>* __restrict__ B, cx<R>* __restrict__ grid, int64_t grs,
                                     int nrhs, int tile) {
    using C = cx<R>;
    using Wt = typename std::conditional<USEB, C, R>::type;
    constexpr int SP1_CAP = sp1_cap<Wt, C, W, RC>();
    __shared__ Wt s_w[SP1_CAP][W];
    __shared__ C s_f[SP1_CAP][RC];
    __shared__ int s_rel[SP1_CAP];
    __shared__ int s_pos[SP1_TS + 2 * MAX_M_CUT + 1];
    const int Ms = g.Ms[0], m2 = 2 * g.m;
    const int TS = min(SP1_TS, Ms - m2);          // the window c0-2m .. c0+TS-1 never wraps onto itself
    const int c0 = tile * TS;
    if (c0 >= Ms) return;
    const int hi = min(c0 + TS, Ms);
    const int nrel = hi - c0 + m2;                  // relative cells 0 .. nrel-1
    const Tile1 T(nd, c0, m2, Ms);
    for (int r = threadIdx.x; r <= nrel; r += blockDim.x) s_pos[r] = T.pos(nd, r);
    __syncthreads();
    const int ntot = s_pos[nrel];
    const int t = threadIdx.x;
    const bool own = t < hi - c0;
    const int a = own ? s_pos[t] : 0, b = own ? s_pos[t + m2 + 1] : 0;   // this cell's node range
    for (int r0 = 0; r0 < nrhs; r0 += RC) {
        const int rc = min(RC, nrhs - r0);
        C acc[RC];
#pragma unroll
        for (int q = 0; q < RC; ++q) acc[q] = cmake((R)0, (R)0);
        for (int k0 = 0; k0 < ntot; k0 += SP1_CAP) {
            const int nk = min(SP1_CAP, ntot - k0);
            __syncthreads();   // the previous chunk is consumed
            for (int i = threadIdx.x; i < nk; i += blockDim.x) {
                const int p = T.sorted(k0 + i);
                int rel = nd.l0s[p] - T.lo;
                if (rel >= Ms) rel -= Ms;
                if (rel < 0) rel += Ms;
                s_rel[i] = rel;
                const int j = nd.perm[p];
#pragma unroll
                for (int q = 0; q < RC; ++q)
                    if (q < rc) s_f[i][q] = f[(int64_t)(r0 + q) * g.N + j];
                if constexpr (USEB) {
#pragma unroll
                    for (int tau = 0; tau < W; ++tau) s_w[i][tau] = B[(int64_t)tau * g.N + p];
                } else {
                    R wv[W];
                    window_row<R, W>(g, nd.us[p], wv);
#pragma unroll
                    for (int tau = 0; tau < W; ++tau) s_w[i][tau] = wv[tau];
                }
            }
            __syncthreads();
            if (own) {
                const int ia = max(a - k0, 0), ib = min(b - k0, nk);
                for (int i = ia; i < ib; ++i) {
                    const int tau = t + m2 - s_rel[i];
                    const Wt w = s_w[i][tau];
#pragma unroll
                    for (int q = 0; q < RC; ++q) {
                        if constexpr (USEB) acc[q] = cadd(acc[q], cmulc(s_f[i][q], w));
                        else acc[q] = cadd(acc[q], cscale(s_f[i][q], w));
                    }
                }
            }
        }
        if (own) {
#pragma unroll
            for (int q = 0; q < RC; ++q)
                if (q < rc) grid[(int64_t)(r0 + q) * grs + c0 + t] = acc[q];
        }
    }
}

template <typename R, int W, bool USEB, int RC>
__global__ void __launch_bounds__(SP1_TS) k_spread1d(Geo g, NodesDev nd, const cx<R>* __restrict__ f,
                                                     const cx<R>* __restrict__ B, cx<R>* __restrict__ grid,
                                                     int64_t grs, int nrhs) {
    spread1d_tile<R, W, USEB, RC>(g, nd, f, B, grid, grs, nrhs, blockIdx.x);
}

template <typename R, int W, bool USEB, int RC>
__global__ void __launch_bounds__(SP1_TS) k_spread1d_batched(const NodeJob* __restrict__ jobs,
                                                             const int2* __restrict__ bmap, const cx<R>* f,
                                                             int nrhs) {
    const int2 bm = bmap[blockIdx.x];
    const NodeJob& J = jobs[bm.x];
    spread1d_tile<R, W, USEB, RC>(J.g, J.nd, f + (int64_t)nrhs * J.noff, (const cx<R>*)J.B, (cx<R>*)J.grid, J.grs,
                                  nrhs, bm.y);
}

int spread1d_tiles(const Geo& g) {
    const int TS = std::min(SP1_TS, g.Ms[0] - 2 * g.m);
    return (g.Ms[0] + TS - 1) / TS;
}

// ------------------------------------------------------------------ gradient with respect to x

template <typename R, int D, int W>
__device__ inline void grad_x_item(const Geo& g, const NodesDev& nd, const cx<R>* __restrict__ grid, int64_t grs,
                                   const cx<R>* __restrict__ gradf, double* __restrict__ gradx, int nrhs,
                                   int accumulate, int64_t j) {
    using C = cx<R>;
    if (j >= g.N) return;
    const R b = (R)g.b;
    R w0[W], w1[W], d0[W], d1[W];
    window_row<R, W>(g, nd.uc[j * D], w0);
    window_deriv_row<R, W>(g, nd.uc[j * D], (R)g.Ms[0], d0);
    const int a0 = nd.l0c[j * D];
    int a1 = 0;
    if (D == 2) {
        window_row<R, W>(g, nd.uc[j * D + 1], w1);
        window_deriv_row<R, W>(g, nd.uc[j * D + 1], (R)g.Ms[1], d1);
        a1 = nd.l0c[j * D + 1];
    }
    R gx0 = 0, gx1 = 0;
    for (int r = 0; r < nrhs; ++r) {
        const C* gr = grid + r * grs;
        C s0 = cmake((R)0, (R)0), s1 = cmake((R)0, (R)0);
        if (D == 1) {
#pragma unroll
            for (int t = 0; t < W; ++t) {
                const C v = gr[wrap_add(a0, t, g.Ms[0])];
                s0.x += d0[t] * v.x;
                s0.y += d0[t] * v.y;
            }
        } else {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                const C* row = gr + (int64_t)wrap_add(a0, t0, g.Ms[0]) * g.Ms[1];
                C sw = cmake((R)0, (R)0), sd = cmake((R)0, (R)0);
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const C v = row[wrap_add(a1, t1, g.Ms[1])];
                    sw.x += w1[t1] * v.x;
                    sw.y += w1[t1] * v.y;
                    sd.x += d1[t1] * v.x;
                    sd.y += d1[t1] * v.y;
                }
                s0.x += d0[t0] * sw.x;
                s0.y += d0[t0] * sw.y;
                s1.x += w0[t0] * sd.x;
                s1.y += w0[t0] * sd.y;
            }
        }
        const C gf = gradf[r * g.N + j];
        gx0 += gf.x * s0.x + gf.y * s0.y;
        if (D == 2) gx1 += gf.x * s1.x + gf.y * s1.y;
    }
    if (accumulate) {
        gradx[j * D] += (double)gx0;
        if (D == 2) gradx[j * D + 1] += (double)gx1;
    } else {
        gradx[j * D] = (double)gx0;
        if (D == 2) gradx[j * D + 1] = (double)gx1;
    }
}

template <typename R, int D, int W>
__global__ void __launch_bounds__(256) k_grad_x(Geo g, NodesDev nd, const cx<R>* __restrict__ grid,
                                                int64_t grs, const cx<R>* __restrict__ gradf,
                                                double* __restrict__ gradx, int nrhs, int accumulate) {
    grad_x_item<R, D, W>(g, nd, grid, grs, gradf, gradx, nrhs, accumulate,
                         blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------------ many 1-D problems in one launch
// Workgroup -> (job, block of that job's items).  A job's caller-side arrays are the batch arrays
// plus nrhs times its node offset (problem-major layout).

template <typename R, int W>
__global__ void __launch_bounds__(256) k_interp_batched(const NodeJob* __restrict__ jobs, const int2* __restrict__ bmap,
                                                        cx<R>* f, int nrhs) {
    const int2 b = bmap[blockIdx.x];
    const NodeJob& J = jobs[b.x];
    interp_item<R, 1, W>(J.g, J.nd, (const cx<R>*)J.grid, J.grs, f + (int64_t)nrhs * J.noff, nrhs,
                         (int64_t)b.y * 256 + threadIdx.x);
}

template <typename R, int W>
__global__ void __launch_bounds__(256) k_interp_B_batched(const NodeJob* __restrict__ jobs,
                                                          const int2* __restrict__ bmap, cx<R>* f, int nrhs) {
    const int2 b = bmap[blockIdx.x];
    const NodeJob& J = jobs[b.x];
    interp_B_item<R, 1, W>(J.g, J.nd, (const cx<R>*)J.grid, J.grs, (const cx<R>*)J.B, f + (int64_t)nrhs * J.noff,
                           nrhs, (int64_t)b.y * 256 + threadIdx.x);
}

template <typename R, int W>
__global__ void __launch_bounds__(256) k_grad_x_batched(const NodeJob* __restrict__ jobs,
                                                        const int2* __restrict__ bmap, const cx<R>* gradf,
                                                        double* gradx, int nrhs, int accumulate) {
    const int2 b = bmap[blockIdx.x];
    const NodeJob& J = jobs[b.x];
    grad_x_item<R, 1, W>(J.g, J.nd, (const cx<R>*)J.grid, J.grs, gradf + (int64_t)nrhs * J.noff, gradx + J.noff,
                         nrhs, accumulate, (int64_t)b.y * 256 + threadIdx.x);
}

// ------------------------------------------------------------------ launchers

#define INFFT_DISPATCH_W(m, ...)                 \
    switch (m) {                                 \
        case 2: { constexpr int W = 5; __VA_ARGS__; } break;  \
        case 3: { constexpr int W = 7; __VA_ARGS__; } break;  \
        case 4: { constexpr int W = 9; __VA_ARGS__; } break;  \
        case 5: { constexpr int W = 11; __VA_ARGS__; } break; \
        case 6: { constexpr int W = 13; __VA_ARGS__; } break; \
        case 7: { constexpr int W = 15; __VA_ARGS__; } break; \
        default: { constexpr int W = 17; __VA_ARGS__; } break; \
    }

// right-hand sides per pass of the tiled 1-D spreading (1, 2, 4 or 8), window or B_opt weights
#define INFFT_SPREAD1D_RC(useb, nrhs, ...)                                              \
    if (nrhs >= 8) { constexpr int RC = 8; constexpr bool USEB = useb; __VA_ARGS__; }   \
    else if (nrhs >= 4) { constexpr int RC = 4; constexpr bool USEB = useb; __VA_ARGS__; } \
    else if (nrhs >= 2) { constexpr int RC = 2; constexpr bool USEB = useb; __VA_ARGS__; } \
    else { constexpr int RC = 1; constexpr bool USEB = useb; __VA_ARGS__; }
#define INFFT_SPREAD1D_DISPATCH(nrhs, m, useB, ...)                                  \
    if (useB) { INFFT_DISPATCH_W(m, INFFT_SPREAD1D_RC(true, nrhs, __VA_ARGS__)) }      \
    else { INFFT_DISPATCH_W(m, INFFT_SPREAD1D_RC(false, nrhs, __VA_ARGS__)) }

template <typename R>
void launch_interp(const Geo& g, NodesDev nd, const cx<R>* grid, int64_t grs, cx<R>* f, int nrhs,
                   hipStream_t s) {
    const unsigned blocks = (unsigned)((g.N + 255) / 256);
    if (g.d == 1) {
        INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_interp<R, 1, W>), dim3(blocks), dim3(256), 0, s, g, nd,
                                                 grid, grs, f, nrhs))
    } else {
        INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_interp<R, 2, W>), dim3(blocks), dim3(256), 0, s, g, nd,
                                                 grid, grs, f, nrhs))
    }
}

template <typename R>
void launch_interp_B(const Geo& g, NodesDev nd, const cx<R>* grid, int64_t grs, const cx<R>* B, cx<R>* f,
                     int nrhs, hipStream_t s) {
    const unsigned blocks = (unsigned)((g.N + 255) / 256);
    if (g.d == 1) {
        INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_interp_B<R, 1, W>), dim3(blocks), dim3(256), 0, s, g,
                                                 nd, grid, grs, B, f, nrhs))
    } else {
        INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_interp_B<R, 2, W>), dim3(blocks), dim3(256), 0, s, g,
                                                 nd, grid, grs, B, f, nrhs))
    }
}

int spread_rhs_chunk(const Geo& g) {
    const int64_t cells = (int64_t)(g.TS[0] + 2 * g.m) * (g.d == 2 ? g.TS[1] + 2 * g.m : 1);
    const int64_t per = cells * 2 * (int64_t)sizeof(double);
    int rc = (int)((48 * 1024) / per);
    if (rc < 1) rc = 1;
    if (rc > 16) rc = 16;
    return rc;
}

template <typename R>
void launch_spread(const Geo& g, NodesDev nd, const cx<R>* f, const cx<R>* B, cx<R>* grid, int64_t grs,
                   cx<R>* h0, cx<R>* h1, cx<R>* h01, int64_t hrs0, int64_t hrs1, int64_t hrs01, int nrhs,
                   int rchunk, SpreadWork wk, hipStream_t s) {
    if (g.d == 1) {
        // right-hand sides per pass: the largest power of two up to min(nrhs, rchunk, 8)
        const dim3 nb(spread1d_tiles(g)), bl(SP1_TS);
        const int rcap = rchunk > 0 ? min(nrhs, rchunk) : nrhs;
        INFFT_SPREAD1D_DISPATCH(rcap, g.m, B != nullptr,
                                hipLaunchKernelGGL((k_spread1d<R, W, USEB, RC>), nb, bl, 0, s, g, nd, f, B, grid, grs,
                                                   nrhs))
        return;
    }
    const unsigned ntiles = (unsigned)(g.ntile[0] * g.ntile[1]);
    hipLaunchKernelGGL(k_spread_zero_split<R>, dim3(ntiles), dim3(256), 0, s, g, wk, grid, grs, h0, h1, h01, hrs0,
                       hrs1, hrs01, nrhs);
    const unsigned blocks = (unsigned)wk.cap;
    const int64_t cells = (int64_t)(g.TS[0] + 2 * g.m) * (g.d == 2 ? g.TS[1] + 2 * g.m : 1);
    const int rc = min(rchunk, nrhs);
    const size_t shm = (size_t)rc * cells * 2 * sizeof(double);
    const unsigned nrc = (unsigned)((nrhs + rc - 1) / rc);
#define INFFT_SPREAD(D_, USEB_)                                                                   \
    INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_spread<R, D_, W, USEB_>), dim3(blocks, nrc), dim3(256), shm, s, \
                                             g, nd, f, B, grid, grs, h0, h1, h01, hrs0, hrs1, hrs01, nrhs, rc, wk))
    if (B) { INFFT_SPREAD(2, true) } else { INFFT_SPREAD(2, false) }
#undef INFFT_SPREAD
}

template <typename R>
void launch_grad_x(const Geo& g, NodesDev nd, const cx<R>* grid, int64_t grs, const cx<R>* gradf,
                   double* gradx, int nrhs, int accumulate, hipStream_t s) {
    const unsigned blocks = (unsigned)((g.N + 255) / 256);
    if (g.d == 1) {
        INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_grad_x<R, 1, W>), dim3(blocks), dim3(256), 0, s, g, nd,
                                                 grid, grs, gradf, gradx, nrhs, accumulate))
    } else {
        INFFT_DISPATCH_W(g.m, hipLaunchKernelGGL((k_grad_x<R, 2, W>), dim3(blocks), dim3(256), 0, s, g, nd,
                                                 grid, grs, gradf, gradx, nrhs, accumulate))
    }
}

template <typename R>
void launch_node_batched(int kind, int m, const NodeJob* jobs, const int2* bmap, int nblocks, const cx<R>* in,
                         cx<R>* out, double* gradx, int nrhs, int accumulate, hipStream_t s) {
    if (nblocks <= 0) return;
    const dim3 gr(nblocks), bl(256);
    switch (kind) {
        case NB_INTERP:
            INFFT_DISPATCH_W(m, hipLaunchKernelGGL((k_interp_batched<R, W>), gr, bl, 0, s, jobs, bmap, out, nrhs))
            break;
        case NB_INTERP_B:
            INFFT_DISPATCH_W(m, hipLaunchKernelGGL((k_interp_B_batched<R, W>), gr, bl, 0, s, jobs, bmap, out, nrhs))
            break;
        case NB_GATHER:
        case NB_GATHER_B: {
            const dim3 sb(SP1_TS);
            INFFT_SPREAD1D_DISPATCH(nrhs, m, kind == NB_GATHER_B,
                                    hipLaunchKernelGGL((k_spread1d_batched<R, W, USEB, RC>), gr, sb, 0, s, jobs, bmap,
                                                       in, nrhs))
            break;
        }
        default:
            INFFT_DISPATCH_W(m, hipLaunchKernelGGL((k_grad_x_batched<R, W>), gr, bl, 0, s, jobs, bmap, in, gradx,
                                                   nrhs, accumulate))
            break;
    }
}

#define INFFT_INST(R)                                                                                  \
    template void launch_interp<R>(const Geo&, NodesDev, const cx<R>*, int64_t, cx<R>*, int, hipStream_t); \
    template void launch_interp_B<R>(const Geo&, NodesDev, const cx<R>*, int64_t, const cx<R>*, cx<R>*, int, \
                                     hipStream_t);                                                     \
    template void launch_spread<R>(const Geo&, NodesDev, const cx<R>*, const cx<R>*, cx<R>*, int64_t, cx<R>*, \
                                   cx<R>*, cx<R>*, int64_t, int64_t, int64_t, int, int, SpreadWork,    \
                                   hipStream_t);                                                       \
    template void launch_grad_x<R>(const Geo&, NodesDev, const cx<R>*, int64_t, const cx<R>*, double*, int, \
                                   int, hipStream_t);                                                  \
    template void launch_node_batched<R>(int, int, const NodeJob*, const int2*, int, const cx<R>*, cx<R>*,    \
                                         double*, int, int, hipStream_t);
INFFT_INST(float)
INFFT_INST(double)

}  // namespace infft
