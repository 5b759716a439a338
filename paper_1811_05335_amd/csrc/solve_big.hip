// Local least-squares problems of Algorithm 3.17 with more members than one lane group holds
// (FP64): the dense centre of polar and spiral trajectories gives |I(l)| in the thousands.
//
// The system is the same as in the register tiers: (G + lambda I) b = r with
// G[i][j] = M_sigma^d Q(z_j - z_i) and r_i = conj K(z_i), z = tau - u per dimension.  Here G is
// formed in device memory (row-major, lower triangle) and factorised by a blocked right-looking
// Cholesky with 64 x 64 blocks.  The host has read the problem sizes back, sorted the problems
// by size (largest first) and packed them into batches whose matrices fit the workspace.  Per
// batch:
//   k_big_setup   one workgroup per problem: members of I(l), z, r and the tap of each member
//   k_big_gram    one workgroup per 64 x 64 tile of the lower triangle
//   for each block column k:
//     k_big_potrf   factor the diagonal block in LDS and invert the factor (lower triangular)
//     k_big_trsm    panel below it: L[i][k] = A[i][k] L_kk^{-*} (a product with the inverse)
//     k_big_herk    trailing tiles: A[i][j] -= L[i][k] L[j][k]^*, k < j <= i (FP64 matrix cores)
//   k_big_solve   L y = r and L^* b = y with the inverse diagonal blocks, b written to B_opt
// The inverse X = L_kk^{-1} needs no storage of its own: its strictly lower part, conjugated and
// transposed, fills the unused strictly upper part of the diagonal block, and X[i][i] = 1/L[i][i].
// Problems sorted largest first make "problems with more than k block columns" a prefix of the
// batch, so k_big_potrf needs no task list.
#include "internal.hpp"

namespace infft {

constexpr int CELL_TPB = 128;
constexpr int MAX_CELLS = (2 * MAX_M_CUT + 1) * (2 * MAX_M_CUT + 1);

// Cell c of the (2m+1)^d cells whose nodes may reach grid index l: the CSR range of its nodes
// and whether it sits at tap 2m in a dimension (there only nodes with u at m reach l).
__device__ inline void big_cell(const Geo& g, const NodesDev& nd, int l, int c, int& s, int& e, bool& edge0,
                                bool& edge1) {
    const int W = 2 * g.m + 1, w2 = 2 * g.m;
    if (g.d == 1) {
        int c0 = l - c;
        if (c0 < 0) c0 += g.Ms[0];
        s = nd.start[c0];
        e = nd.start[c0 + 1];
        edge0 = c == w2;
        edge1 = false;
    } else {
        const int lc0 = l / g.Ms[1], lc1 = l - lc0 * g.Ms[1];
        const int tau0 = c / W, tau1 = c - tau0 * W;
        int c0 = lc0 - tau0;
        if (c0 < 0) c0 += g.Ms[0];
        int c1 = lc1 - tau1;
        if (c1 < 0) c1 += g.Ms[1];
        const int64_t key = cell_key(g, c0, c1);
        s = nd.start[key];
        e = nd.start[key + 1];
        edge0 = tau0 == w2;
        edge1 = tau1 == w2;
    }
}

__device__ inline bool big_member(const Geo& g, const NodesDev& nd, int p, bool edge0, bool edge1) {
    if (edge0 && !edge_tap_member(nd.us[(int64_t)p * g.d], g.m)) return false;
    if (edge1 && !edge_tap_member(nd.us[(int64_t)p * g.d + 1], g.m)) return false;
    return true;
}

__device__ inline int big_cell_count(const Geo& g, const NodesDev& nd, int l, int c) {
    int s, e;
    bool e0, e1;
    big_cell(g, nd, l, c, s, e, e0, e1);
    if (!e0 && !e1) return e - s;
    int n = 0;
    for (int p = s; p < e; ++p) n += big_member(g, nd, p, e0, e1) ? 1 : 0;
    return n;
}

__device__ inline int num_cells(const Geo& g) {
    const int W = 2 * g.m + 1;
    return g.d == 1 ? W : W * W;
}

// |I(l)| for each listed grid index.
__global__ void __launch_bounds__(CELL_TPB) k_big_count(Geo g, NodesDev nd, const int* __restrict__ list,
                                                        int* __restrict__ nout) {
    __shared__ int s_sum[CELL_TPB];
    const int l = list[blockIdx.x];
    int n = 0;
    for (int c = threadIdx.x; c < num_cells(g); c += CELL_TPB) n += big_cell_count(g, nd, l, c);
    s_sum[threadIdx.x] = n;
    __syncthreads();
    for (int w = CELL_TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) nout[blockIdx.x] = s_sum[0];
}

void launch_big_count(const Geo& g, NodesDev nd, const int* list, int count, int* nout, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_big_count, dim3(count), dim3(CELL_TPB), 0, s, g, nd, list, nout);
}

// Members of one problem (cells in order, nodes of a cell in sorted order), then per member the
// tap index, z = tau - u per dimension and r = conj K(z).
__global__ void __launch_bounds__(CELL_TPB) k_big_setup(Geo g, NodesDev nd, KTabDev kt, BigArgs a) {
    if (a.stale && *a.stale) return;
    __shared__ int s_base[MAX_CELLS + 1];
    const BigProb P = a.probs[blockIdx.x];
    const int ncell = num_cells(g);
    for (int c = threadIdx.x; c < ncell; c += CELL_TPB) s_base[c + 1] = big_cell_count(g, nd, P.l, c);
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base[0] = 0;
        for (int c = 0; c < ncell; ++c) s_base[c + 1] += s_base[c];
        if (s_base[ncell] != P.n) a.fail[P.id] = 2;   // cannot happen: the count uses the same test
    }
    __syncthreads();
    if (s_base[ncell] != P.n) return;
    int* midx = a.midx + P.moff;
    for (int c = threadIdx.x; c < ncell; c += CELL_TPB) {
        int s, e;
        bool e0, e1;
        big_cell(g, nd, P.l, c, s, e, e0, e1);
        int pos = s_base[c];
        for (int p = s; p < e && pos < P.n; ++p)
            if (big_member(g, nd, p, e0, e1)) midx[pos++] = p;
    }
    __syncthreads();
    const int W = 2 * g.m + 1;
    int lc0 = P.l, lc1 = 0;
    if (g.d == 2) {
        lc0 = P.l / g.Ms[1];
        lc1 = P.l - lc0 * g.Ms[1];
    }
    for (int i = threadIdx.x; i < P.n; i += CELL_TPB) {
        const int p = midx[i];
        int tau0 = lc0 - nd.l0s[(int64_t)p * g.d];
        if (tau0 < 0) tau0 += g.Ms[0];
        double2 z = make_double2((double)tau0 - nd.us[(int64_t)p * g.d], 0.0);
        double2 K = tay_eval(kt.K[0], kt.qK, z.x);
        int tap = tau0;
        if (g.d == 2) {
            int tau1 = lc1 - nd.l0s[(int64_t)p * 2 + 1];
            if (tau1 < 0) tau1 += g.Ms[1];
            z.y = (double)tau1 - nd.us[(int64_t)p * 2 + 1];
            K = cmul(K, tay_eval(kt.K[1], kt.qK, z.y));
            tap = tau0 * W + tau1;
        }
        a.mtap[P.moff + i] = tap;
        a.mz[P.moff + i] = z;
        a.mr[P.moff + i] = cconj(K);
    }
}

void launch_big_setup(const Geo& g, NodesDev nd, KTabDev kt, BigArgs a, int nprob, hipStream_t s) {
    if (nprob <= 0) return;
    hipLaunchKernelGGL(k_big_setup, dim3(nprob), dim3(CELL_TPB), 0, s, g, nd, kt, a);
}

// Tile (I, J), J <= I, of the lower triangle of G + lambda I.
__global__ void __launch_bounds__(BIG_TPB) k_big_gram(Geo g, KTabDev kt, BigArgs a, const int4* __restrict__ tasks) {
    if (a.stale && *a.stale) return;
    __shared__ double2 s_zi[BIG_NB];
    const int4 t = tasks[blockIdx.x];
    const BigProb P = a.probs[t.x];
    const int i0 = t.y * BIG_NB, j0 = t.z * BIG_NB;
    if (threadIdx.x < BIG_NB) {
        const int i = i0 + threadIdx.x;
        s_zi[threadIdx.x] = i < P.n ? a.mz[P.moff + i] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int j = j0 + (threadIdx.x & (BIG_NB - 1));
    if (j >= P.n) return;
    const double2 zj = a.mz[P.moff + j];
    double2* A = a.A + P.off;
    for (int rr = threadIdx.x / BIG_NB; rr < BIG_NB; rr += BIG_TPB / BIG_NB) {
        const int i = i0 + rr;
        if (i >= P.n || j > i) continue;
        const double2 zi = s_zi[rr];
        double2 v = tay_eval(kt.Q[0], kt.qQ, zj.x - zi.x);
        if (g.d == 2) v = cmul(v, tay_eval(kt.Q[1], kt.qQ, zj.y - zi.y));
        v = cscale(v, kt.scaleG);
        if (i == j) v = make_double2(v.x + kt.lam, 0.0);
        A[(int64_t)i * P.n + j] = v;
    }
}

void launch_big_gram(const Geo& g, KTabDev kt, BigArgs a, const int4* tasks, int ntask, hipStream_t s) {
    if (ntask <= 0) return;
    hipLaunchKernelGGL(k_big_gram, dim3(ntask), dim3(BIG_TPB), 0, s, g, kt, a, tasks);
}

// Diagonal block k of problem blockIdx.x: Cholesky in LDS, then X = L_kk^{-1} row by row
// (X[i][j] = (delta_ij - sum_{j<=q<i} L[i][q] X[q][j]) / L[i][i]).  A non-positive pivot marks
// the problem failed (its later steps run on zeros and its solution is not written).
__global__ void __launch_bounds__(BIG_TPB) k_big_potrf(BigArgs a, int k) {
    if (a.stale && *a.stale) return;
    // L in the lower triangle of T; the inverse X, conjugated, in its strictly upper triangle
    // (T[j][i] = conj X[i][j], i > j), so that two workgroups fit a CU
    __shared__ double2 T[BIG_NB][BIG_NB + 1];
    __shared__ double2 red[BIG_TPB / BIG_NB][BIG_NB];
    const BigProb P = a.probs[blockIdx.x];
    const int r0 = k * BIG_NB, nk = min(BIG_NB, P.n - r0);
    double2* D = a.A + P.off + (int64_t)r0 * P.n + r0;   // the diagonal block
    const int64_t ld = P.n;
    for (int e = threadIdx.x; e < BIG_NB * BIG_NB; e += BIG_TPB) {
        const int i = e / BIG_NB, j = e % BIG_NB;
        T[i][j] = (i < nk && j <= i) ? D[(int64_t)i * ld + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    bool ok = true;
    for (int c = 0; c < nk; ++c) {
        const double piv = T[c][c].x;   // the same value in every thread: the exit is uniform
        if (!(piv > 0.0) || !isfinite(piv)) {
            ok = false;
            break;
        }
        const double sq = sqrt(piv), inv = 1.0 / sq;
        __syncthreads();
        if (threadIdx.x == 0) T[c][c] = make_double2(sq, 0.0);
        for (int i = c + 1 + threadIdx.x; i < nk; i += BIG_TPB) T[i][c] = cscale(T[i][c], inv);
        __syncthreads();
        const int w = nk - c - 1;
        for (int e = threadIdx.x; e < w * w; e += BIG_TPB) {
            const int i = c + 1 + e / w, j = c + 1 + e % w;
            if (j <= i) T[i][j] = csub(T[i][j], cmulc(T[i][c], T[j][c]));
        }
        __syncthreads();
    }
    if (ok) {
        // row i of X from the rows before it: X[q][j] = conj T[j][q] for q > j, 1/L[j][j] for q = j
        const int j = threadIdx.x % BIG_NB, part = threadIdx.x / BIG_NB;
        constexpr int NP = BIG_TPB / BIG_NB;
        for (int i = 1; i < nk; ++i) {
            double2 acc = make_double2(0.0, 0.0);
            if (j < i) {
                for (int q = j + part; q < i; q += NP) {
                    const double2 xq = q == j ? make_double2(1.0 / T[j][j].x, 0.0) : cconj(T[j][q]);
                    acc = cadd(acc, cmul(T[i][q], xq));
                }
            }
            red[part][j] = acc;
            __syncthreads();
            if (part == 0 && j < i) {
                double2 s = red[0][j];
                for (int pp = 1; pp < NP; ++pp) s = cadd(s, red[pp][j]);
                T[j][i] = cconj(cscale(s, -1.0 / T[i][i].x));
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < BIG_NB * BIG_NB; e += BIG_TPB) {
        const int i = e / BIG_NB, j = e % BIG_NB;
        if (i >= nk || j >= nk) continue;
        if (j <= i) D[(int64_t)i * ld + j] = T[i][j];
        else D[(int64_t)i * ld + j] = ok ? T[i][j] : make_double2(0.0, 0.0);
    }
    if (!ok && threadIdx.x == 0) a.fail[P.id] = 1;
}

void launch_big_potrf(BigArgs a, int nprob, int k, hipStream_t s) {
    if (nprob <= 0) return;
    hipLaunchKernelGGL(k_big_potrf, dim3(nprob), dim3(BIG_TPB), 0, s, a, k);
}

// Register tile of a 64 x 64 complex product: thread (tr, tc) owns rows 4 tr .. 4 tr + 3 and
// columns 4 tc .. 4 tc + 3.
struct Tile4 {
    double2 v[4][4];
    __device__ void zero() {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[a][b] = make_double2(0.0, 0.0);
    }
    // v += x y^*
    __device__ void acc(const double2 (&x)[4], const double2 (&y)[4]) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                v[a][b].x = fma(x[a].x, y[b].x, fma(x[a].y, y[b].y, v[a][b].x));
                v[a][b].y = fma(x[a].y, y[b].x, fma(-x[a].x, y[b].y, v[a][b].y));
            }
    }
};

// Panel block (I, k): A[I][k] <- A[I][k] X^*, X = L_kk^{-1}.
__global__ void __launch_bounds__(BIG_TPB) k_big_trsm(BigArgs a, const int4* __restrict__ tasks, int k) {
    if (a.stale && *a.stale) return;
    constexpr int KC = 16;
    __shared__ double2 sA[KC][BIG_NB + 1];   // [q][row]
    __shared__ double2 sX[KC][BIG_NB + 1];   // [q][col]
    const int4 t = tasks[blockIdx.x];
    const BigProb P = a.probs[t.x];
    const int r0 = t.y * BIG_NB, c0 = k * BIG_NB;
    const int nr = min(BIG_NB, P.n - r0), nk = min(BIG_NB, P.n - c0);
    double2* A = a.A + P.off;
    const int64_t ld = P.n;
    const double2* D = A + (int64_t)c0 * ld + c0;
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
    Tile4 acc;
    acc.zero();
    for (int q0 = 0; q0 < nk; q0 += KC) {
#pragma unroll
        for (int s = 0; s < BIG_NB * KC / BIG_TPB; ++s) {
            const int e = threadIdx.x + s * BIG_TPB;
            const int r = e / KC, qq = e % KC, q = q0 + qq;
            sA[qq][r] = (r < nr && q < nk) ? A[(int64_t)(r0 + r) * ld + c0 + q] : make_double2(0.0, 0.0);
            sX[qq][r] = (r < nk && q < nk) ? inv_entry(D, ld, r, q) : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int qq = 0; qq < KC; ++qq) {
            double2 x[4], y[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                x[u] = sA[qq][tr * 4 + u];
                y[u] = sX[qq][tc * 4 + u];
            }
            acc.acc(x, y);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = tr * 4 + u, c = tc * 4 + v;
            if (r < nr && c < nk) A[(int64_t)(r0 + r) * ld + c0 + c] = acc.v[u][v];
        }
}

void launch_big_trsm(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s) {
    if (ntask <= 0) return;
    hipLaunchKernelGGL(k_big_trsm, dim3(ntask), dim3(BIG_TPB), 0, s, a, tasks, k);
}

// Trailing tile (I, J), k < J <= I: A[I][J] -= L[I][k] L[J][k]^* (lower part only when I == J), on
// the FP64 matrix cores: C = L[I][k] L[J][k]^* as four real products, Re C = Ar Jr^T + Ai Ji^T and
// Im C = Ai Jr^T - Ar Ji^T, with v_mfma_f64_16x16x4.  Each wavefront owns a 32 x 32 quadrant of the
// 64 x 64 tile (2 x 2 blocks of 16 x 16).  Operand layout of the instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result element i of lane l is C[l / 16 + 4 i][l % 16].
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(BIG_TPB) k_big_herk(BigArgs a, const int4* __restrict__ tasks, int k) {
    if (a.stale && *a.stale) return;
    constexpr int KC = 16;
    __shared__ double2 sI[KC][BIG_NB + 1];
    __shared__ double2 sJ[KC][BIG_NB + 1];
    const int4 t = tasks[blockIdx.x];
    const BigProb P = a.probs[t.x];
    const int rI = t.y * BIG_NB, rJ = t.z * BIG_NB, c0 = k * BIG_NB;
    const int nI = min(BIG_NB, P.n - rI), nJ = min(BIG_NB, P.n - rJ), nk = min(BIG_NB, P.n - c0);
    double2* A = a.A + P.off;
    const int64_t ld = P.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;   // quadrant of this wavefront
    const int lr = lane & 15, lk = lane >> 4;
    v4d cr[2][2], ci[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            cr[u][v] = v4d{0.0, 0.0, 0.0, 0.0};
            ci[u][v] = v4d{0.0, 0.0, 0.0, 0.0};
        }
    // the next chunk is loaded into registers while the current one is multiplied
    constexpr int PER = BIG_NB * KC / BIG_TPB;
    double2 nxI[PER], nxJ[PER];
    auto fetch = [&](int q0) {
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int e = threadIdx.x + s * BIG_TPB;
            const int r = e / KC, qq = e % KC, q = q0 + qq;
            nxI[s] = (r < nI && q < nk) ? A[(int64_t)(rI + r) * ld + c0 + q] : make_double2(0.0, 0.0);
            nxJ[s] = (r < nJ && q < nk) ? A[(int64_t)(rJ + r) * ld + c0 + q] : make_double2(0.0, 0.0);
        }
    };
    fetch(0);
    for (int q0 = 0; q0 < nk; q0 += KC) {
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int e = threadIdx.x + s * BIG_TPB;
            const int r = e / KC, qq = e % KC;
            sI[qq][r] = nxI[s];
            sJ[qq][r] = nxJ[s];
        }
        __syncthreads();
        if (q0 + KC < nk) fetch(q0 + KC);
#pragma unroll
        for (int qs = 0; qs < KC; qs += 4) {
            double ar[2], ai[2], jr[2], ji[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double2 x = sI[qs + lk][wr + 16 * u + lr];
                ar[u] = x.x;
                ai[u] = x.y;
                const double2 y = sJ[qs + lk][wc + 16 * u + lr];
                jr[u] = y.x;
                ji[u] = y.y;
            }
            // consecutive instructions update different accumulators
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    cr[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[u], jr[v], cr[u][v], 0, 0, 0);
                    ci[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[u], jr[v], ci[u][v], 0, 0, 0);
                }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    cr[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[u], ji[v], cr[u][v], 0, 0, 0);
                    ci[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[u], ji[v], ci[u][v], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    const bool diag = t.y == t.z;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = wr + 16 * u + lk + 4 * i, c = wc + 16 * v + lr;
                if (r < nI && c < nJ && (!diag || c <= r)) {
                    double2* dst = &A[(int64_t)(rI + r) * ld + rJ + c];
                    *dst = csub(*dst, make_double2(cr[u][v][i], ci[u][v][i]));
                }
            }
}

void launch_big_herk(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s) {
    if (ntask <= 0) return;
    hipLaunchKernelGGL(k_big_herk, dim3(ntask), dim3(BIG_TPB), 0, s, a, tasks, k);
}

// Forward and backward substitution for one problem, then its column of B_opt.  The right-hand
// side vector is overwritten by y and then by b; the workgroup's own global writes are visible
// to its threads after each barrier.
__global__ void __launch_bounds__(BIG_TPB) k_big_solve(Geo g, BigArgs a, double2* __restrict__ B64,
                                                       float2* __restrict__ B32) {
    if (a.stale && *a.stale) return;
    const BigProb P = a.probs[blockIdx.x];
    const int fl = a.fail[P.id];   // 1: non-positive pivot (zero column written), 2: no members known
    if (fl == 2) return;
    const double2* A = a.A + P.off;
    double2* y = a.mr + P.moff;
    const int nblk = fl ? 0 : P.nblk;
    big_substitute(P, A, y, nblk);
    for (int i = threadIdx.x; i < P.n; i += BIG_TPB) {
        const int64_t idx = (int64_t)a.mtap[P.moff + i] * g.N + a.midx[P.moff + i];
        const double2 b = fl ? make_double2(0.0, 0.0) : y[i];
        put_bopt(B64, B32, idx, b);
    }
}

void launch_big_solve(const Geo& g, BigArgs a, int nprob, double2* B64, float2* B32, hipStream_t s) {
    if (nprob <= 0) return;
    hipLaunchKernelGGL(k_big_solve, dim3(nprob), dim3(BIG_TPB), 0, s, g, a, B64, B32);
}

// The same two substitutions spread over the whole GPU, one launch per block step (right-looking):
// a problem of n = 5000 members holds 200 MB of factor, which one workgroup reads at a fraction of
// HBM bandwidth.  Forward step k, per task (problem, I >= k): y_k = X_k r_k (X_k = L_kk^{-1}, every
// task recomputes it from r_k, which no task of step k writes); task I = k stores y_k, tasks I > k
// update r_I -= L[I][k] y_k.  Backward step k, per task (problem, J <= k): b_k = X_k^* y_k; task J = k
// stores b_k over r_k, tasks J < k update y_J -= L[k][J]^* b_k.  r lives in mr, y in mb.
__device__ inline void big_block_vec(const double2* D, int64_t ld, int nk, const double2* v, double2* out,
                                     bool adjoint, double2 (&red)[BIG_TPB / BIG_NB][BIG_NB]) {
    // out = X v (adjoint: X^* v) for the inverse X of the diagonal block D; 64 x 64, in LDS
    constexpr int NP = BIG_TPB / BIG_NB;
    const int c = threadIdx.x % BIG_NB, part = threadIdx.x / BIG_NB;
    double2 acc = make_double2(0.0, 0.0);
    if (c < nk) {
        if (!adjoint) {
            for (int q = part; q <= c; q += NP) acc = cadd(acc, cmul(inv_entry(D, ld, c, q), v[q]));
        } else {
            for (int q = c + part; q < nk; q += NP) acc = cadd(acc, cmul(cconj(inv_entry(D, ld, q, c)), v[q]));
        }
    }
    red[part][c] = acc;
    __syncthreads();
    if (part == 0) {
        double2 sum = red[0][c];
        for (int pp = 1; pp < NP; ++pp) sum = cadd(sum, red[pp][c]);
        out[c] = c < nk ? sum : make_double2(0.0, 0.0);
    }
    __syncthreads();
}

__global__ void __launch_bounds__(BIG_TPB) k_big_fwd(BigArgs a, const int4* __restrict__ tasks, int k) {
    if (a.stale && *a.stale) return;
    constexpr int NP = BIG_TPB / BIG_NB;
    __shared__ double2 s_r[BIG_NB], s_y[BIG_NB];
    __shared__ double2 red[NP][BIG_NB];
    const int4 t = tasks[blockIdx.x];
    const BigProb P = a.probs[t.x];
    if (a.fail[P.id]) return;
    const int64_t ld = P.n;
    const int r0 = k * BIG_NB, nk = min(BIG_NB, P.n - r0);
    const double2* A = a.A + P.off;
    double2* r = a.mr + P.moff;
    double2* y = a.mb + P.moff;
    if (threadIdx.x < BIG_NB) s_r[threadIdx.x] = threadIdx.x < nk ? r[r0 + threadIdx.x] : make_double2(0.0, 0.0);
    __syncthreads();
    big_block_vec(A + (int64_t)r0 * ld + r0, ld, nk, s_r, s_y, false, red);
    if (t.y == k) {
        if (threadIdx.x < nk) y[r0 + threadIdx.x] = s_y[threadIdx.x];
        return;
    }
    // r_I -= L[I][k] y_k: NP threads per row
    const int I0 = t.y * BIG_NB, nr = min(BIG_NB, P.n - I0);
    const int row = threadIdx.x / NP, p4 = threadIdx.x % NP;
    double2 acc = make_double2(0.0, 0.0);
    if (row < nr) {
        const double2* Lr = A + (int64_t)(I0 + row) * ld + r0;
        for (int c = p4; c < nk; c += NP) acc = cadd(acc, cmul(Lr[c], s_y[c]));
    }
#pragma unroll
    for (int o = 1; o < NP; o <<= 1) {
        acc.x += __shfl_xor(acc.x, o, 64);
        acc.y += __shfl_xor(acc.y, o, 64);
    }
    if (p4 == 0 && row < nr) r[I0 + row] = csub(r[I0 + row], acc);
}

__global__ void __launch_bounds__(BIG_TPB) k_big_bwd(BigArgs a, const int4* __restrict__ tasks, int k) {
    if (a.stale && *a.stale) return;
    constexpr int NP = BIG_TPB / BIG_NB;
    __shared__ double2 s_v[BIG_NB], s_b[BIG_NB];
    __shared__ double2 red[NP][BIG_NB];
    const int4 t = tasks[blockIdx.x];
    const BigProb P = a.probs[t.x];
    if (a.fail[P.id]) return;
    const int64_t ld = P.n;
    const int r0 = k * BIG_NB, nk = min(BIG_NB, P.n - r0);
    const double2* A = a.A + P.off;
    double2* b = a.mr + P.moff;
    double2* y = a.mb + P.moff;
    if (threadIdx.x < BIG_NB) s_v[threadIdx.x] = threadIdx.x < nk ? y[r0 + threadIdx.x] : make_double2(0.0, 0.0);
    __syncthreads();
    big_block_vec(A + (int64_t)r0 * ld + r0, ld, nk, s_v, s_b, true, red);
    if (t.y == k) {
        if (threadIdx.x < nk) b[r0 + threadIdx.x] = s_b[threadIdx.x];
        return;
    }
    // y_J -= L[k][J]^* b_k: column col of block (k, J), rows summed in NP parts
    const int J0 = t.y * BIG_NB;
    const int col = threadIdx.x % BIG_NB, part = threadIdx.x / BIG_NB;
    double2 acc = make_double2(0.0, 0.0);
    for (int c = part; c < nk; c += NP) acc = cadd(acc, cmul(cconj(A[(int64_t)(r0 + c) * ld + J0 + col]), s_b[c]));
    red[part][col] = acc;
    __syncthreads();
    if (part == 0) {
        double2 sum = red[0][col];
        for (int pp = 1; pp < NP; ++pp) sum = cadd(sum, red[pp][col]);
        y[J0 + col] = csub(y[J0 + col], sum);
    }
}

// The solutions into B_opt (zeros for failed problems; nothing for problems without members).
__global__ void __launch_bounds__(BIG_TPB) k_big_write(Geo g, BigArgs a, double2* __restrict__ B64,
                                                       float2* __restrict__ B32) {
    if (a.stale && *a.stale) return;
    const BigProb P = a.probs[blockIdx.x];
    const int fl = a.fail[P.id];
    if (fl == 2) return;
    const double2* b = a.mr + P.moff;
    for (int i = threadIdx.x; i < P.n; i += BIG_TPB) {
        const int64_t idx = (int64_t)a.mtap[P.moff + i] * g.N + a.midx[P.moff + i];
        const double2 v = fl ? make_double2(0.0, 0.0) : b[i];
        put_bopt(B64, B32, idx, v);
    }
}

void launch_big_fwd(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s) {
    if (ntask <= 0) return;
    hipLaunchKernelGGL(k_big_fwd, dim3(ntask), dim3(BIG_TPB), 0, s, a, tasks, k);
}

void launch_big_bwd(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s) {
    if (ntask <= 0) return;
    hipLaunchKernelGGL(k_big_bwd, dim3(ntask), dim3(BIG_TPB), 0, s, a, tasks, k);
}

void launch_big_write(const Geo& g, BigArgs a, int nprob, double2* B64, float2* B32, hipStream_t s) {
    if (nprob <= 0) return;
    hipLaunchKernelGGL(k_big_write, dim3(nprob), dim3(BIG_TPB), 0, s, g, a, B64, B32);
}

// One statistics record for the whole pass: sizes known on the host, failures counted here.
__global__ void __launch_bounds__(256) k_big_stats(const int* fail, int n, int nmin, int nmax, long long* rec) {
    __shared__ int sh[256];
    int f = 0;
    for (int i = threadIdx.x; i < n; i += 256) f += fail[i] ? 1 : 0;
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rec[0] = nmin;
        rec[1] = nmax;
        rec[2] = sh[0];
        rec[3] = 0;
        rec[4] = 0;
    }
}

void launch_big_stats(const int* fail, int n, int nmin, int nmax, long long* rec, hipStream_t s) {
    hipLaunchKernelGGL(k_big_stats, dim3(1), dim3(256), 0, s, fail, n, nmin, nmax, rec);
}


// ------------------------------------------------------------------ recorded problems under capture

__global__ void k_big_slots(const BigProb* __restrict__ probs, int count, int* __restrict__ slot) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) slot[probs[i].l] = i;
}

void launch_big_slots(const BigProb* probs, int count, int* slot, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_big_slots, dim3((count + 255) / 256), dim3(256), 0, s, probs, count, slot);
}

constexpr int CHECK_BLOCKS = 256;

__global__ void __launch_bounds__(CELL_TPB) k_big_check(Geo g, NodesDev nd, const int* __restrict__ list,
                                                        const int* __restrict__ count, const int* __restrict__ slot,
                                                        const BigProb* __restrict__ probs, int rec_count, int gen,
                                                        int* __restrict__ stale) {
    __shared__ int s_sum[CELL_TPB];
    const int cnt = *count;
    if (stale[1] != gen) {   // a newer record replaced the one this launch was made for
        if (blockIdx.x == 0 && threadIdx.x == 0) stale[0] = 1;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && cnt != rec_count) stale[0] = 1;
    const int lim = min(cnt, rec_count);
    for (int i = blockIdx.x; i < lim; i += gridDim.x) {
        const int l = list[i];
        int n = 0;
        for (int c = threadIdx.x; c < num_cells(g); c += CELL_TPB) n += big_cell_count(g, nd, l, c);
        s_sum[threadIdx.x] = n;
        __syncthreads();
        for (int w = CELL_TPB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int k = slot[l];
            if (k < 0 || k >= rec_count || probs[k].n != s_sum[0]) stale[0] = 1;
        }
        __syncthreads();
    }
}

void launch_big_check(const Geo& g, NodesDev nd, const int* list, const int* count, const int* slot,
                      const BigProb* probs, int rec_count, int gen, int* stale, hipStream_t s) {
    hipLaunchKernelGGL(k_big_check, dim3(CHECK_BLOCKS), dim3(CELL_TPB), 0, s, g, nd, list, count, slot, probs,
                       rec_count, gen, stale);
}

// Zeroes the B_opt entries of the listed problems and counts them as oversized.
// The count goes to statistics record 0, which nfft_plan_status folds into the status block, and
// to the status word itself, which the host reads as is when it has not seen a precompute since
// its last nfft_set_nodes (a replayed graph does not tell the host).
__device__ inline void big_zero_listed(const Geo& g, const NodesDev& nd, const int* __restrict__ list, int cnt,
                                       double2* __restrict__ B64, float2* __restrict__ B32, long long* rec0,
                                       long long* status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rec0[4] = cnt;
        status[ST_OVERSIZED] = cnt;
    }
    if (g.d != 1) return;   // 2-D columns were cleared before the tiers ran
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int l = list[i];
        for (int c = 0; c < num_cells(g); ++c) {
            int st, e;
            bool e0, e1;
            big_cell(g, nd, l, c, st, e, e0, e1);
            for (int q = st + (int)threadIdx.x; q < e; q += CELL_TPB) {
                if (!big_member(g, nd, q, e0, e1)) continue;
                int tau = l - nd.l0s[q];
                if (tau < 0) tau += g.Ms[0];
                const int64_t idx = (int64_t)tau * g.N + q;
                put_bopt(B64, B32, idx, make_double2(0.0, 0.0));
            }
        }
    }
}

__global__ void __launch_bounds__(CELL_TPB) k_big_zero_stale(Geo g, NodesDev nd, const int* __restrict__ list,
                                                             const int* __restrict__ count,
                                                             const int* __restrict__ stale, double2* __restrict__ B64,
                                                             float2* __restrict__ B32, long long* rec0,
                                                             long long* status) {
    if (!*stale) return;
    big_zero_listed(g, nd, list, *count, B64, B32, rec0, status);
}

__global__ void __launch_bounds__(CELL_TPB) k_big_guard_empty(Geo g, NodesDev nd, const int* __restrict__ list,
                                                              const int* __restrict__ count,
                                                              const int* __restrict__ gen_dev, int gen,
                                                              double2* __restrict__ B64, float2* __restrict__ B32,
                                                              long long* rec0, long long* status) {
    const int cnt = *count;
    if (cnt == 0 && *gen_dev == gen) return;
    big_zero_listed(g, nd, list, cnt, B64, B32, rec0, status);
}

void launch_big_guard_empty(const Geo& g, NodesDev nd, const int* list, const int* count, const int* gen_dev, int gen,
                            double2* B64, float2* B32, long long* rec0, long long* status, hipStream_t s) {
    hipLaunchKernelGGL(k_big_guard_empty, dim3(CHECK_BLOCKS), dim3(CELL_TPB), 0, s, g, nd, list, count, gen_dev, gen,
                       B64, B32, rec0, status);
}

void launch_big_zero_stale(const Geo& g, NodesDev nd, const int* list, const int* count, const int* stale,
                           double2* B64, float2* B32, long long* rec0, long long* status, hipStream_t s) {
    hipLaunchKernelGGL(k_big_zero_stale, dim3(CHECK_BLOCKS), dim3(CELL_TPB), 0, s, g, nd, list, count, stale, B64,
                       B32, rec0, status);
}

}  // namespace infft
