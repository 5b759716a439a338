// Batched local least-squares problems of Algorithm 3.17 (FP64).
//
// For every oversampled grid index l the optimised column of B solves (3.29)-(3.31) with a ridge:
//     b_l = argmin || L_l b - e_l ||^2 + lambda ||b||^2,   L_l[s, j] = K(s/M_sigma - x_j)  (3.30)
// The paper evaluates L_l (M_sigma^d rows) with one NFFT per l.  Here the normal equations are
// formed directly: since F has orthogonal columns, sum_s e^{2 pi i (k'-k) s / M_sigma} =
// M_sigma delta_{kk'} for |k - k'| < M_sigma, so
//     (L_l^* L_l)[i, j] = M_sigma^d Q(x_i - x_j),      Q(y) = sum_k D_k^2 e^{2 pi i k.y}
//     (L_l^* e_l)[j]     = conj K(l/M_sigma - x_j),     K(y) = sum_k D_k   e^{2 pi i k.y}
// (tensor products over dimensions).  In grid units both arguments are small: with the tap
// tau_j = (l - l0_j) mod M_sigma and z_j = tau_j - u_j in [-m, m], K is needed at z_j and Q at
// z_j - z_i in [-2m, 2m]; both come from the Taylor tables built at plan time.
//
// Layout of the work.  1-D: a thread per grid index up to 13 members (the band of a workgroup's
// node range in LDS); then groups of 16 lanes, one or two rows of the real system per lane in
// registers, reduced by Gaussian elimination with DPP broadcasts (up to 16 or 32 members); then a
// wavefront with the matrix in LDS (up to 64).  2-D: a group of NL lanes (NL = 16 or 32) owns one
// grid index at a time; the members of I(l) are gathered from the (2m+1)^2 grid cells whose nodes
// reach l (the node CSR); lane i owns member i and row i of the Hermitian system, and the Cholesky
// factorisation, forward and backward substitution pass each step's column or partial sums
// through a small per-thread LDS slot, so all reads of a step issue together.  Problems beyond a
// tier's size are passed on to the next tier.
#include "internal.hpp"

#include <limits.h>
#include <utility>

namespace infft {

// Copies n doubles from global memory to LDS with the whole workgroup, eight loads in flight per
// thread before the first store.
__device__ inline void stage_to_lds(double* dst, const double* __restrict__ src, int n) {
    for (int i0 = threadIdx.x; i0 < n; i0 += 8 * blockDim.x) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = i0 + k * blockDim.x;
            v[k] = (i < n) ? glb(src)[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = i0 + k * blockDim.x;
            if (i < n) dst[i] = v[k];
        }
    }
}


// Per-block statistics of the solve kernels.  Each block reduces its waves' counters and writes
// one record with plain stores (same-address global atomics from every wave would serialise in
// the L2); k_solve_stats folds the records into the status block once all tiers have run.
struct SolveStat {
    unsigned long long mn, mx, fail, empty, over;
};

__device__ inline void write_block_stats(long long* rec, int64_t blk, unsigned long long st_min, unsigned long long st_max,
                                         unsigned long long st_fail, unsigned long long st_empty,
                                         unsigned long long st_over) {
    __shared__ SolveStat s_st[16];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        st_min = min(st_min, (unsigned long long)__shfl_xor((long long)st_min, o, 64));
        st_max = max(st_max, (unsigned long long)__shfl_xor((long long)st_max, o, 64));
        st_fail += (unsigned long long)__shfl_xor((long long)st_fail, o, 64);
        st_empty += (unsigned long long)__shfl_xor((long long)st_empty, o, 64);
        st_over += (unsigned long long)__shfl_xor((long long)st_over, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_st[w] = SolveStat{st_min, st_max, st_fail, st_empty, st_over};
    __syncthreads();
    if (threadIdx.x == 0) {
        SolveStat t = s_st[0];
        for (int i = 1; i < (int)(blockDim.x + 63) / 64; ++i) {
            t.mn = min(t.mn, s_st[i].mn);
            t.mx = max(t.mx, s_st[i].mx);
            t.fail += s_st[i].fail;
            t.empty += s_st[i].empty;
            t.over += s_st[i].over;
        }
        long long* r = rec + blk * 5;
        r[0] = (long long)t.mn;
        r[1] = (long long)t.mx;
        r[2] = (long long)t.fail;
        r[3] = (long long)t.empty;
        r[4] = (long long)t.over;
    }
}

// First tier of a B optimisation: statistics record 0 (the large-problem guard's) back to "no
// problem, nothing oversized".
__device__ inline void reset_rec0(const SolveArgs& a) {
    if (a.rec0 && blockIdx.x == 0 && threadIdx.x < 5) a.rec0[threadIdx.x] = (threadIdx.x == 0) ? -1LL : 0;
}

// The list counters start at zero without a reset launch: each launch of a B optimisation clears,
// from workgroup 0, counters that no kernel reads any more and a later launch appends to.
__device__ inline void clear_counters(const SolveArgs& a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (a.zero0) *a.zero0 = 0;
        if (a.zero1) *a.zero1 = 0;
    }
}

__global__ void __launch_bounds__(256) k_solve_stats(const long long* rec, int nrec, long long* status) {
    __shared__ unsigned long long sh[5][256];
    unsigned long long mn = ULLONG_MAX, mx = 0, fail = 0, empty = 0, over = 0;
    for (int i = threadIdx.x; i < nrec; i += blockDim.x) {
        mn = min(mn, (unsigned long long)rec[i * 5 + 0]);
        mx = max(mx, (unsigned long long)rec[i * 5 + 1]);
        fail += rec[i * 5 + 2];
        empty += rec[i * 5 + 3];
        over += rec[i * 5 + 4];
    }
    sh[0][threadIdx.x] = mn;
    sh[1][threadIdx.x] = mx;
    sh[2][threadIdx.x] = fail;
    sh[3][threadIdx.x] = empty;
    sh[4][threadIdx.x] = over;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            sh[0][threadIdx.x] = min(sh[0][threadIdx.x], sh[0][o]);
            sh[1][threadIdx.x] = max(sh[1][threadIdx.x], sh[1][o]);
            sh[2][threadIdx.x] += sh[2][o];
            sh[3][threadIdx.x] += sh[3][o];
            sh[4][threadIdx.x] += sh[4][o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        status[ST_MIN_N] = (sh[0][0] == ULLONG_MAX) ? LLONG_MAX : (long long)sh[0][0];
        status[ST_MAX_N] = (long long)sh[1][0];
        status[ST_FAILED] = (long long)sh[2][0];
        status[ST_EMPTY] = (long long)sh[3][0];
        status[ST_OVERSIZED] = (long long)sh[4][0];
    }
}

void launch_solve_stats(const long long* rec, int nrec, long long* status, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_stats, dim3(1), dim3(256), 0, s, rec, nrec, status);
}

template <int D, int NL>
__device__ inline void solve_group_body(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a);

template <int D, int NL>
__global__ void __launch_bounds__(256) k_solve(Geo g, NodesDev nd, KTabDev kt, SolveArgs a) {
    reset_rec0(a);
    clear_counters(a);
    solve_group_body<D, NL>(g, nd, kt, a);
}

template <int D, int NL>
__device__ inline void solve_group_body(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a) {
    __shared__ double2 s_col[256];   // per-thread exchange slot (column broadcasts, reductions)
    __shared__ double2 s_z[256];     // z of each member (x: dimension 0, y: dimension 1)
    extern __shared__ double2 s_tab[];
    const int lane = threadIdx.x & (NL - 1);
    const int sb = threadIdx.x - lane;               // first slot of this group
    const int gbase = (threadIdx.x & 63) - lane;     // first lane of this group inside the wave
    const uint64_t gmask = (NL == 64) ? ~0ull : ((1ull << NL) - 1ull);
    const int64_t gid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / NL;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / NL;
    const int64_t count = a.in_list ? (int64_t)(*a.in_count) : g.G;
    const int W = 2 * g.m + 1;

    // 1-D plans keep the Q table (read n times per member) in LDS; K is read once per member.
    const double2* tK0 = kt.K[0];
    const double2* tQ0 = kt.Q[0];
    if (D == 1 && a.tables_in_lds) {
        const int nQ = (kt.qQ + 1) * TAY_NC;
        for (int i = threadIdx.x; i < nQ; i += blockDim.x) s_tab[i] = kt.Q[0][i];
        __syncthreads();
        tQ0 = s_tab;
    }

    unsigned long long st_min = ULLONG_MAX, st_max = 0, st_fail = 0, st_empty = 0, st_over = 0;

    for (int64_t qi = gid; qi < count; qi += ngroups) {
        const int l = a.in_list ? glb(a.in_list)[qi] : (int)qi;
        int n = 0, my_p = 0;
        if (D == 1) gather_1d(g, nd, l, lane, NL, gbase, gmask, n, my_p);
        else gather_2d(g, nd, l, lane, NL, gbase, gmask, n, my_p);
        if (n == 0) {
            if (lane == 0) ++st_empty;
            continue;
        }
        if (n > NL) {
            if (lane == 0) {
                if (a.out_list) {
                    const int slot = atomicAdd(a.out_count, 1);
                    a.out_list[slot] = l;
                } else {
                    ++st_over;
                }
            }
            continue;
        }
        if (lane == 0) {
            st_min = min(st_min, (unsigned long long)n);
            st_max = max(st_max, (unsigned long long)n);
        }
        const bool act = lane < n;

        // ---- tap tau = (l - l0) mod M_sigma and z = tau - u per dimension; r = conj K(z)
        double z0 = 0.0, z1 = 0.0;
        int my_tau = 0;
        double2 y = make_double2(0.0, 0.0);
        if (act) {
            if (D == 1) {
                int tau0 = l - glb(nd.l0s)[my_p];
                if (tau0 < 0) tau0 += g.Ms[0];
                z0 = (double)tau0 - glb(nd.us)[my_p];
                my_tau = tau0;
                y = cconj(tay_eval(tK0, kt.qK, z0));
            } else {
                const int lc0 = l / g.Ms[1], lc1 = l - lc0 * g.Ms[1];
                int tau0 = lc0 - glb(nd.l0s)[(int64_t)my_p * 2];
                if (tau0 < 0) tau0 += g.Ms[0];
                int tau1 = lc1 - glb(nd.l0s)[(int64_t)my_p * 2 + 1];
                if (tau1 < 0) tau1 += g.Ms[1];
                z0 = (double)tau0 - glb(nd.us)[(int64_t)my_p * 2];
                z1 = (double)tau1 - glb(nd.us)[(int64_t)my_p * 2 + 1];
                my_tau = tau0 * W + tau1;
                y = cconj(cmul(tay_eval(kt.K[0], kt.qK, z0), tay_eval(kt.K[1], kt.qK, z1)));
            }
        }
        s_z[threadIdx.x] = make_double2(z0, z1);
        wave_sync();

        // ---- row i of G + lambda I (lower triangle): G[i][j] = M_sigma^d Q(z_j - z_i)
        double2 A[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            A[j] = make_double2(0.0, 0.0);
            if (j < n) {
                const double2 zj = s_z[sb + j];
                double2 qv;
                if (D == 1) qv = tay_eval(tQ0, kt.qQ, zj.x - z0);
                else qv = cmul(tay_eval(kt.Q[0], kt.qQ, zj.x - z0), tay_eval(kt.Q[1], kt.qQ, zj.y - z1));
                A[j] = cscale(qv, kt.scaleG);
                if (j == lane) A[j] = make_double2(A[j].x + kt.lam, 0.0);
            }
        }

        // ---- Cholesky G + lambda I = L L^*, lane i keeps row i of L.  Step k broadcasts the
        // unscaled column k through LDS; with inv = 1/sqrt(pivot) the update of row i is
        // A[i][j] -= (A[i][k] inv^2) conj(A[j][k]) for k < j <= i.
        bool ok = true;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (k < n && ok) {
                s_col[threadIdx.x] = A[k];
                wave_sync();
                const double piv = s_col[sb + k].x;
                ok = piv > 0.0;
                const double sq = sqrt(ok ? piv : 1.0), inv = 1.0 / sq;
                const double2 Lk2 = cscale(A[k], inv * inv);
#pragma unroll
                for (int j = k + 1; j < NL; ++j) {
                    if (j < n) {
                        const double2 raw = s_col[sb + j];
                        if (lane >= j) {
                            A[j].x -= Lk2.x * raw.x + Lk2.y * raw.y;
                            A[j].y -= Lk2.y * raw.x - Lk2.x * raw.y;
                        }
                    }
                }
                if (lane == k) A[k] = make_double2(sq, 0.0);
                else if (lane > k) A[k] = cscale(A[k], inv);
                wave_sync();
            }
        }
        if (!ok) {
            if (lane == 0) ++st_fail;
            continue;
        }

        // ---- forward substitution L y = r
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (k < n) {
                if (lane == k) y = cscale(y, 1.0 / A[k].x);
                s_col[threadIdx.x] = y;
                wave_sync();
                const double2 yk = s_col[sb + k];
                if (lane > k && act) y = csub(y, cmul(A[k], yk));
                wave_sync();
            }
        }
        // ---- backward substitution L^* b = y: b_k = (y_k - sum_{i>k} conj(L[i][k]) b_i) / L[k][k]
        double2 bsol = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = NL - 1; k >= 0; --k) {
            if (k < n) {
                s_col[threadIdx.x] = (lane > k && act) ? cmul(cconj(A[k]), bsol) : make_double2(0.0, 0.0);
                wave_sync();
                if (lane == k) {
                    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
                    for (int j = k + 1; j < NL; ++j) sum = cadd(sum, s_col[sb + j]);
                    bsol = cscale(csub(y, sum), 1.0 / A[k].x);
                }
                wave_sync();
            }
        }

        // ---- scatter into B_opt ([tap][sorted node])
        if (act) {
            const int64_t idx = (int64_t)my_tau * g.N + my_p;
            put_bopt(a.B64, a.B32, idx, bsol);
        }
        wave_sync();
    }

    // ---- statistics: reduce over the wave, one set of atomics per wave
    write_block_stats(a.stat_rec + (int64_t)a.stat_off * 5, blockIdx.x, st_min, st_max, st_fail, st_empty, st_over);
}

// ------------------------------------------------------------------ 1-D: real solves + rank one
// In one dimension the frequencies +-k pair up except k = -M/2, so with d = D_{-M/2},
// w_i = e^{i pi z_i / sigma} and the real, even sums Ks, Qs over the pairs:
//     G + lambda I = A0 + c w w^*,   A0 = M_sigma Qs(z_j - z_i) + lambda I (real SPD),  c = M_sigma d^2
//     r            = Ks(z) + d w
// and the Sherman-Morrison formula gives the solution from three real solves with A0,
//     t = A0^{-1} Ks,  u = A0^{-1} w,  s = w^* u (real, >= 0),
//     b = t + u (d - c w^* t) / (1 + c s),
// whose denominator is at least one.

template <typename P>
__device__ inline double tay_eval_r(P tab, int qmax, double z) {
    const double az = fabs(z);
    int q = (int)rint(az * (double)TAY_S);
    if (q > qmax) q = qmax;
    const double e = az - (double)q * (1.0 / TAY_S);
    const auto c = tab + (int64_t)q * TAY_NC;
    double acc = c[TAY_NC - 1];
#pragma unroll
    for (int p = TAY_NC - 2; p >= 0; --p) acc = fma(acc, e, c[p]);
    return acc;
}

// Entries of B_opt belonging to a 1-D problem that no tier solves are set to zero.
__device__ inline void zero_members_1d(const Geo& g, const NodesDev& nd, int l, int lane, int NL,
                                       const SolveArgs& a) {
    const int Ms = g.Ms[0], w2 = 2 * g.m;
    int lo = l - w2;
    if (lo < 0) lo += Ms;
    for (int c = 0; c <= w2; ++c) {
        int cell = lo + c;
        if (cell >= Ms) cell -= Ms;
        const int s = glb(nd.start)[cell], e = glb(nd.start)[cell + 1];
        for (int p = s + lane; p < e; p += NL) {
            int tau = l - glb(nd.l0s)[p];
            if (tau < 0) tau += Ms;
            put_bopt(a.B64, a.B32, (int64_t)tau * g.N + p, make_double2(0.0, 0.0));
        }
    }
}

template <int NL>
__device__ inline double group_sum(double v) {
#pragma unroll
    for (int o = NL / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Solve statistics of one lane group (accumulated by its lane 0).
struct GroupStats {
    unsigned long long mn = ULLONG_MAX, mx = 0, fail = 0, empty = 0, over = 0;
};

// ---- 16-lane groups: exchanges through DPP within a row of 16 lanes (no LDS, no wave barrier)

// Lane K of the caller's row of 16 lanes, to every lane of that row.
template <int K> __device__ __forceinline__ double row_bcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + K, 0xf, 0xf, true);
}

// Sum over the 16 lanes of a row: two quad permutations, then rotations by 4 and 8 in the row.
__device__ __forceinline__ double row_sum16(double v) {
    v += __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xf, 0xf, true);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xf, 0xf, true);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x124, 0xf, 0xf, true);  // row_ror:4
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x128, 0xf, 0xf, true);  // row_ror:8
    return v;
}

// 1 / x for x > 0: the hardware estimate and two Newton steps r <- r + r (1 - x r).
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// Members of a 1-D problem for a group of 16 lanes holding R rows each: row 16 r + lane is member
// 16 r + lane (the order of gather_1d: the cells l-2m+1 .. l, then the edge-tap members of l-2m).
template <int R>
__device__ __forceinline__ void gather_1d_rows(const Geo& g, const NodesDev& nd, int l, int lane, int gbase, int& n,
                                      int (&my_p)[R]) {
    const int w2 = 2 * g.m, Ms = g.Ms[0];
    const int clo = l - w2 + 1;
    int s0, e0, s1 = 0, e1 = 0;
    if (clo >= 0) {
        s0 = glb(nd.start)[clo];
        e0 = glb(nd.start)[l + 1];
    } else {
        s0 = glb(nd.start)[clo + Ms];
        e0 = glb(nd.start)[Ms];
        s1 = glb(nd.start)[0];
        e1 = glb(nd.start)[l + 1];
    }
    const int n0 = e0 - s0, n1 = e1 - s1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gi = 16 * r + lane;
        my_p[r] = gi < n0 ? s0 + gi : (gi - n0 < n1 ? s1 + (gi - n0) : 0);
    }
    n = n0 + n1;
    int ce = l - w2;
    if (ce < 0) ce += Ms;
    const int s = glb(nd.start)[ce], e = glb(nd.start)[ce + 1];
    for (int base = s; base < e; base += 16) {
        const int p = base + lane;
        const bool mem = p < e && edge_tap_member(glb(nd.us)[p], g.m);
        const uint32_t gm = (uint32_t)(__ballot(mem) >> gbase) & 0xffffu;
        const int cnt = __popc(gm);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = 16 * r + lane - n;
            if (k >= 0 && k < cnt) {
                uint32_t mm = gm;
                for (int i = 0; i < k; ++i) mm &= mm - 1u;
                my_p[r] = base + (__ffs(mm) - 1);
            }
        }
        n += cnt;
    }
}

// The state of one problem on its 16-lane group: R rows per lane (row 16 r + lane) of the real
// system and of the three right-hand sides (Ks, Re w, Im w).  One row per lane keeps full rows;
// with more, row array r keeps columns 0 .. 16 r + 15 (the lower triangle and the rest of its
// block), which the elimination in lower form needs.
template <int R> struct GeRows {
    static constexpr int NC = 16 * R;
    static constexpr bool FULL = R == 1;
    static constexpr int width(int r) { return FULL ? NC : 16 * (r + 1); }
    static constexpr int off(int r) { return FULL ? r * NC : 8 * r * (r + 1); }
    double A[off(R)];
    double t[R], ur[R], ui[R];
    double dinv[R];   // 1 / d of the lane's rows once eliminated
    __device__ __forceinline__ double& a(int r, int j) { return A[off(r) + j]; }
    __device__ __forceinline__ double a(int r, int j) const { return A[off(r) + j]; }
};

// Column J of the lane's rows of A0 = M_sigma Qs(z_j - z_i) + lambda I (identity rows and columns
// past n): the table rows, then the Horner steps.
template <int R, int J, typename TP>
__device__ __forceinline__ void ge_gram_load(const double (&z)[R], const KTabDev& kt, TP tQ,
                                    double (&e)[R], double (&cf)[R][TAY_NC]) {
    const double zj = row_bcast<J % 16>(z[J / 16]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (J >= GeRows<R>::width(r)) continue;
        const double az = fabs(zj - z[r]);
        int q = (int)rint(az * (double)TAY_S);
        if (q > kt.qQ) q = kt.qQ;
        e[r] = az - (double)q * (1.0 / TAY_S);
        const auto c = tQ + (int64_t)q * TAY_NC;
#pragma unroll
        for (int p = 0; p < TAY_NC; ++p) cf[r][p] = c[p];
    }
}

template <int R, int J>
__device__ __forceinline__ void ge_gram_store(GeRows<R>& S, int lane, int n, const KTabDev& kt, const double (&e)[R],
                                     const double (&cf)[R][TAY_NC]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (J >= GeRows<R>::width(r)) continue;
        const int gi = 16 * r + lane;
        double acc = cf[r][TAY_NC - 1];
#pragma unroll
        for (int p = TAY_NC - 2; p >= 0; --p) acc = fma(acc, e[r], cf[r][p]);
        double v = kt.scaleG * acc;
        if (J == gi) v += kt.lam;
        S.a(r, J) = (gi < n && J < n) ? v : (J == gi ? 1.0 : 0.0);
    }
}

// Columns J .. J+JB-1: every table row of the step is loaded before the first Horner step, and no
// later step's loads are hoisted above it (registers).
template <int R, int J, typename TP, int... B>
__device__ __forceinline__ void ge_gram(GeRows<R>& S, const double (&z)[R], int lane, int n, const KTabDev& kt,
                                        TP tQ, std::integer_sequence<int, B...>) {
    double e[sizeof...(B)][R], cf[sizeof...(B)][R][TAY_NC];
    (ge_gram_load<R, J + B>(z, kt, tQ, e[B], cf[B]), ...);
    (ge_gram_store<R, J + B>(S, lane, n, kt, e[B], cf[B]), ...);
    __builtin_amdgcn_sched_barrier(0);
}

template <int R, int JB, typename TP, int... Jb>
__device__ __forceinline__ void ge_gram_all(GeRows<R>& S, const double (&z)[R], int lane, int n, const KTabDev& kt,
                                   TP tQ, std::integer_sequence<int, Jb...>) {
    (ge_gram<R, Jb * JB>(S, z, lane, n, kt, tQ, std::make_integer_sequence<int, JB>{}), ...);
}

// Column J > K of elimination step K (the pivot row's entry a_KJ, then the update of the lane's rows).
template <int R, int K, int J>
__device__ __forceinline__ void ge_elim_col(GeRows<R>& S, const double (&m)[R]) {
    constexpr int RK = K / 16, LK = K % 16;
    double pj;
    if constexpr (GeRows<R>::FULL) pj = row_bcast<LK>(S.a(RK, J));
    else pj = row_bcast<J % 16>(S.a(J / 16, K));
#pragma unroll
    for (int r = RK; r < R; ++r)
        if (J < GeRows<R>::width(r)) S.a(r, J) = fma(-m[r], pj, S.a(r, J));
    // a few pivot-row entries in flight at a time (registers)
    if constexpr (((J - K) & 7) == 0) __builtin_amdgcn_sched_barrier(0);
}

template <int R, int K, int... J>
__device__ __forceinline__ void ge_elim_cols(GeRows<R>& S, const double (&m)[R], std::integer_sequence<int, J...>) {
    (ge_elim_col<R, K, K + 1 + J>(S, m), ...);
}

// Elimination step K: every row i > K loses l_iK = a_iK / a_KK times the pivot row K (the
// multiplier is zero on the other rows, which keeps them), right-hand sides included.  Full rows
// take the pivot row's entries from the pivot lane; in lower form row i takes a_Kj = a_jK from row
// j's lane (the remaining block stays symmetric) and keeps l_iK in place of a_iK.
template <int R, int K>
__device__ __forceinline__ void ge_elim(GeRows<R>& S, int lane, bool& ok) {
    constexpr int NC = 16 * R, RK = K / 16, LK = K % 16;
    const double piv = row_bcast<LK>(S.a(RK, K));
    ok = ok && piv > 0.0;
    const double inv = rcp_refined(piv > 0.0 ? piv : 1.0);
    if (lane == LK) S.dinv[RK] = inv;
    double m[R];
#pragma unroll
    for (int r = RK; r < R; ++r) m[r] = (16 * r + lane > K) ? S.a(r, K) * inv : 0.0;
    ge_elim_cols<R, K>(S, m, std::make_integer_sequence<int, NC - K - 1>{});
    if constexpr (!GeRows<R>::FULL) {
#pragma unroll
        for (int r = RK; r < R; ++r)
            if (16 * r + lane > K) S.a(r, K) = m[r];
    }
    const double pt = row_bcast<LK>(S.t[RK]), pr = row_bcast<LK>(S.ur[RK]), pi = row_bcast<LK>(S.ui[RK]);
#pragma unroll
    for (int r = RK; r < R; ++r) {
        S.t[r] = fma(-m[r], pt, S.t[r]);
        S.ur[r] = fma(-m[r], pr, S.ur[r]);
        S.ui[r] = fma(-m[r], pi, S.ui[r]);
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <int R, int... K>
__device__ __forceinline__ void ge_elim_all(GeRows<R>& S, int lane, bool& ok, std::integer_sequence<int, K...>) {
    (ge_elim<R, K>(S, lane, ok), ...);
}

// Back substitution step K.  Full rows solve U b = z' (U = D L^T): b_K = z'_K / d_K from the
// pivot lane, then every row i < K loses U[i][K] b_K (the lane's own row entry).  Lower form solves
// L^T b = D^{-1} z' (z already scaled): b_K loses the sum over rows j > K of l_jK b_j, a row sum.
template <int R, int K>
__device__ __forceinline__ void ge_back(const GeRows<R>& S, double (&zr)[R], double (&zi)[R], int lane) {
    constexpr int RK = K / 16, LK = K % 16;
    if constexpr (GeRows<R>::FULL) {
        const double br = row_bcast<LK>(zr[RK] * S.dinv[RK]);
        const double bi = row_bcast<LK>(zi[RK] * S.dinv[RK]);
#pragma unroll
        for (int r = 0; r <= RK; ++r) {
            const double u = (r < RK || lane < LK) ? S.a(r, K) : 0.0;
            zr[r] = fma(-u, br, zr[r]);
            zi[r] = fma(-u, bi, zi[r]);
        }
    } else {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int r = RK; r < R; ++r) {
            const double l = (16 * r + lane > K) ? S.a(r, K) : 0.0;
            sr = fma(l, zr[r], sr);
            si = fma(l, zi[r], si);
        }
        sr = row_sum16(sr);
        si = row_sum16(si);
        if (lane == LK) {
            zr[RK] -= sr;
            zi[RK] -= si;
        }
    }
}

template <int R, int... K>
__device__ __forceinline__ void ge_back_all(const GeRows<R>& S, double (&zr)[R], double (&zi)[R], int lane,
                                   std::integer_sequence<int, K...>) {
    (ge_back<R, 16 * R - 1 - K>(S, zr, zi, lane), ...);
}

// One 1-D problem l of up to 16 R members on a group of 16 lanes (GeRows).  Gaussian elimination
// without pivoting (A0 is SPD: A0 = L D L^T) applied to the rows and the right-hand sides together
// leaves U = D L^T in the rows and y = L^{-1} r in the right-hand sides; the Sherman-Morrison sums
// are then y^T D^{-1} y' and the solution comes from one back substitution with U, each step reading
// the lane's own row.  Every exchange is a DPP broadcast from the pivot lane; rows past n are padded
// with the identity.  A problem with more than 16 R members goes to a.out_list, or without one is
// counted as oversized and its column zeroed.
template <int R, typename TP>
__device__ __forceinline__ void r1_problem_ge(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a, int l,
                                     TP tQ, GroupStats& st) {
    constexpr int NC = 16 * R;
    const int lane = threadIdx.x & 15;
    const int gbase = (threadIdx.x & 63) - lane;
    const double c1 = (double)g.Ms[0] * kt.dM * kt.dM;
    int n = 0, my_p[R];
    gather_1d_rows<R>(g, nd, l, lane, gbase, n, my_p);
    if (n == 0) {
        if (lane == 0) ++st.empty;
        return;
    }
    if (n > NC) {
        if (lane == 0) {
            if (a.out_list) {
                const int slot = atomicAdd(a.out_count, 1);
                a.out_list[slot] = l;
            } else {
                ++st.over;
            }
        }
        if (!a.out_list) zero_members_1d(g, nd, l, lane, 16, a);
        return;
    }
    if (lane == 0) {
        st.mn = min(st.mn, (unsigned long long)n);
        st.mx = max(st.mx, (unsigned long long)n);
    }

    // ---- member data: tap tau, z = tau - u, Ks(z), w = e^{i pi z / sigma}
    GeRows<R> S;
    double z[R];
    int tau[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        z[r] = S.t[r] = S.ur[r] = S.ui[r] = 0.0;
        S.dinv[r] = 1.0;
        tau[r] = 0;
        if (16 * r + lane < n) {
            int tr = l - glb(nd.l0s)[my_p[r]];
            if (tr < 0) tr += g.Ms[0];
            tau[r] = tr;
            z[r] = (double)tr - glb(nd.us)[my_p[r]];
            S.t[r] = tay_eval_r(glb(kt.Ks), kt.qK, z[r]);
            sincospi(z[r] * kt.inv_sigma, &S.ui[r], &S.ur[r]);
        }
    }
    constexpr int JB = R == 1 ? 4 : 1;   // columns per Gram step (4 or 2 table rows in flight)
    ge_gram_all<R, JB>(S, z, lane, n, kt, tQ, std::make_integer_sequence<int, NC / JB>{});

    bool ok = true;
    ge_elim_all<R>(S, lane, ok, std::make_integer_sequence<int, NC>{});
    if (!ok) {
        if (lane == 0) ++st.fail;
        return;
    }

    // ---- Sherman-Morrison: s = w^* A0^{-1} w and w^* A0^{-1} Ks, each a sum y^T D^{-1} y'
    double ps = 0.0, pr = 0.0, pi = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ps = fma(S.dinv[r], fma(S.ur[r], S.ur[r], S.ui[r] * S.ui[r]), ps);
        pr = fma(S.dinv[r], S.ur[r] * S.t[r], pr);
        pi = fma(-S.dinv[r], S.ui[r] * S.t[r], pi);
    }
    const double sdot = row_sum16(ps), wtr = row_sum16(pr), wti = row_sum16(pi);
    const double den = 1.0 + c1 * sdot;
    const double cr = (kt.dM - c1 * wtr) / den, ci = (-c1 * wti) / den;
    // z' = y_k + c' y_w, then the back substitution from the last row up (b = U^{-1} z' with full
    // rows, b = L^{-T} D^{-1} z' in lower form)
    constexpr bool FULL = GeRows<R>::FULL;
    double zr[R], zi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        zr[r] = S.t[r] + cr * S.ur[r] - ci * S.ui[r];
        zi[r] = cr * S.ui[r] + ci * S.ur[r];
        if (!FULL) {
            zr[r] *= S.dinv[r];
            zi[r] *= S.dinv[r];
        }
    }
    ge_back_all<R>(S, zr, zi, lane, std::make_integer_sequence<int, NC>{});
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (16 * r + lane < n) {
            const int64_t idx = (int64_t)tau[r] * g.N + my_p[r];
            const double sc = FULL ? S.dinv[r] : 1.0;
            put_bopt(a.B64, a.B32, idx, make_double2(zr[r] * sc, zi[r] * sc));
        }
    }
}

// The same problem with the group's (n x n) matrix in LDS at Ag, row i of lane i at Ai (wide
// groups: 64 rows in registers would spill); s_y / s_z are the workgroup's exchange slots.
template <int NL, typename TP>
__device__ inline void r1_problem_lds(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a,
                                      int l, TP tQ, double* Ag, double* Ai,
                                      double (*s_y)[128], double* s_z, GroupStats& st) {
    constexpr int LDA = NL + 1;
    const int lane = threadIdx.x & (NL - 1);
    const int sb = threadIdx.x - lane;
    const int gbase = (threadIdx.x & 63) - lane;
    const uint64_t gmask = (NL == 64) ? ~0ull : ((1ull << NL) - 1ull);
    const double c1 = (double)g.Ms[0] * kt.dM * kt.dM;
    int n = 0, my_p = 0;
    gather_1d(g, nd, l, lane, NL, gbase, gmask, n, my_p);
    if (n == 0) {
        if (lane == 0) ++st.empty;
        return;
    }
    if (n > NL) {
        if (lane == 0) {
            if (a.out_list) {
                const int slot = atomicAdd(a.out_count, 1);
                a.out_list[slot] = l;
            } else {
                ++st.over;
            }
        }
        if (!a.out_list) zero_members_1d(g, nd, l, lane, NL, a);
        return;
    }
    if (lane == 0) {
        st.mn = min(st.mn, (unsigned long long)n);
        st.mx = max(st.mx, (unsigned long long)n);
    }
    const bool act = lane < n;

    double z = 0.0, t = 0.0, wr = 0.0, wi = 0.0;
    int tau = 0;
    if (act) {
        tau = l - glb(nd.l0s)[my_p];
        if (tau < 0) tau += g.Ms[0];
        z = (double)tau - glb(nd.us)[my_p];
        t = tay_eval_r(glb(kt.Ks), kt.qK, z);
        sincospi(z * kt.inv_sigma, &wi, &wr);
    }
    double ur = wr, ui = wi;
    s_z[threadIdx.x] = z;
    wave_sync();

    // ---- lower triangle of A0 = M_sigma Qs(z_j - z_i) + lambda I, row i by lane i
    if (act) {
        for (int j0 = 0; j0 <= lane; j0 += 4) {
            double e[4], cf[4][TAY_NC];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double az = fabs(s_z[sb + min(j0 + k, lane)] - z);
                int q = (int)rint(az * (double)TAY_S);
                if (q > kt.qQ) q = kt.qQ;
                e[k] = az - (double)q * (1.0 / TAY_S);
                const auto c = tQ + (int64_t)q * TAY_NC;
#pragma unroll
                for (int p = 0; p < TAY_NC; ++p) cf[k][p] = c[p];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double acc = cf[k][TAY_NC - 1];
#pragma unroll
                for (int p = TAY_NC - 2; p >= 0; --p) acc = fma(acc, e[k], cf[k][p]);
                if (j0 + k <= lane) Ai[j0 + k] = kt.scaleG * acc;
            }
        }
        Ai[lane] += kt.lam;
    }
    wave_sync();

    // ---- Cholesky A0 = L L^T in place (right-looking)
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        const double piv = Ag[k * LDA + k];
        if (!(piv > 0.0)) {
            ok = false;
            break;
        }
        const double sq = sqrt(piv);
        double lik = 0.0;
        if (lane == k) Ai[k] = sq;
        else if (lane > k && act) {
            lik = Ai[k] / sq;
            Ai[k] = lik;
        }
        wave_sync();
        if (lane > k && act)
            for (int j = k + 1; j <= lane; ++j) Ai[j] = fma(-lik, Ag[j * LDA + k], Ai[j]);
        wave_sync();
    }
    if (!ok) {
        if (lane == 0) ++st.fail;
        wave_sync();
        return;
    }

    // ---- forward substitution L y = rhs (Ks, Re w, Im w)
    for (int k = 0; k < n; ++k) {
        if (lane == k) {
            const double iv = 1.0 / Ai[k];
            t *= iv;
            ur *= iv;
            ui *= iv;
            s_y[0][threadIdx.x] = t;
            s_y[1][threadIdx.x] = ur;
            s_y[2][threadIdx.x] = ui;
        }
        wave_sync();
        if (lane > k && act) {
            const double lk = Ai[k];
            t = fma(-lk, s_y[0][sb + k], t);
            ur = fma(-lk, s_y[1][sb + k], ur);
            ui = fma(-lk, s_y[2][sb + k], ui);
        }
    }
    wave_sync();
    // ---- backward substitution L^T x = y
    for (int k = n - 1; k >= 0; --k) {
        if (lane == k) {
            const double iv = 1.0 / Ai[k];
            t *= iv;
            ur *= iv;
            ui *= iv;
            s_y[0][threadIdx.x] = t;
            s_y[1][threadIdx.x] = ur;
            s_y[2][threadIdx.x] = ui;
        }
        wave_sync();
        if (lane < k) {
            const double lk = Ag[k * LDA + lane];
            t = fma(-lk, s_y[0][sb + k], t);
            ur = fma(-lk, s_y[1][sb + k], ur);
            ui = fma(-lk, s_y[2][sb + k], ui);
        }
    }

    // ---- Sherman-Morrison combination
    const double sdot = group_sum<NL>(act ? wr * ur + wi * ui : 0.0);        // w^* u
    const double wtr = group_sum<NL>(act ? wr * t : 0.0);                     // Re w^* t
    const double wti = group_sum<NL>(act ? -wi * t : 0.0);                    // Im w^* t
    const double den = 1.0 + c1 * sdot;
    const double cr = (kt.dM - c1 * wtr) / den, ci = (-c1 * wti) / den;
    const double2 bsol = make_double2(t + ur * cr - ui * ci, ur * ci + ui * cr);

    if (act) {
        const int64_t idx = (int64_t)tau * g.N + my_p;
        put_bopt(a.B64, a.B32, idx, bsol);
    }
    wave_sync();
}

// One problem of up to CAP members: 16-lane groups with CAP / 16 rows per lane up to 32 members
// (registers, DPP exchanges), a 64-lane group with the matrix in LDS beyond (64 rows would not fit
// the registers).  s_A holds the LDS matrices of the workgroup's groups (unused below 64).
template <int CAP> constexpr int group_lanes() { return CAP <= 32 ? 16 : CAP; }

template <int CAP, typename TP>
__device__ inline void r1_solve(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a, int l,
                                TP tQ, double* s_A, double (*s_x)[128], double* s_z, GroupStats& st) {
    if constexpr (CAP > 32) {
        double* Ag = s_A + (threadIdx.x / CAP) * CAP * (CAP + 1);
        r1_problem_lds<CAP>(g, nd, kt, a, l, tQ, Ag, Ag + (threadIdx.x & (CAP - 1)) * (CAP + 1), s_x, s_z, st);
    } else {
        r1_problem_ge<CAP / 16>(g, nd, kt, a, l, tQ, st);
    }
}

// One group of NL lanes per grid index l (r1_solve), over a list or over all grid indices.
// blk / nblk: this workgroup's index and the number of workgroups sharing the problem list.
// TAB_LDS: the Q table is staged in LDS (one problem per launch) or read through the caches.
template <int NL, bool TAB_LDS>
__device__ inline void solve_r1_body(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a,
                                     int64_t blk, int64_t nblk) {
    constexpr int GL = group_lanes<NL>();
    constexpr int GPB = 128 / GL;   // groups per block
    __shared__ double s_A[NL > 32 ? GPB * NL * (NL + 1) : 1];
    __shared__ double s_x[NL > 32 ? 3 : 1][128];
    __shared__ double s_z[NL > 32 ? 128 : 1];
    extern __shared__ double s_tabr[];
    const int64_t gid = (blk * (int64_t)blockDim.x + threadIdx.x) / GL;
    const int64_t ngroups = nblk * blockDim.x / GL;
    const int64_t count = a.in_list ? (int64_t)(*a.in_count) : g.G;
    if (blk * (int64_t)GPB >= count) {
        // no problem for this workgroup (a short list): skip the table staging, leave a neutral record
        write_block_stats(a.stat_rec + (int64_t)a.stat_off * 5, blk, ULLONG_MAX, 0, 0, 0, 0);
        return;
    }

    const double* tQ = kt.Qs;
    if (TAB_LDS) {
        stage_to_lds(s_tabr, kt.Qs, (kt.qQ + 1) * TAY_NC);
        __syncthreads();
        tQ = s_tabr;
    }
    GroupStats st;
    for (int64_t qi = gid; qi < count; qi += ngroups) {
        const int l = a.in_list ? glb(a.in_list)[qi] : (int)qi;
        r1_solve<NL>(g, nd, kt, a, l, tQ, s_A, s_x, s_z, st);
    }
    write_block_stats(a.stat_rec + (int64_t)a.stat_off * 5, blk, st.mn, st.mx, st.fail, st.empty, st.over);
}

// The list of problems of 17 to 64 members (single 1-D plans): each wave takes four entries at a
// time, one per 16-lane group; those of up to 32 members are solved at once by their group (two
// rows per lane), the larger ones afterwards one at a time by the whole wave with the matrix in
// LDS.  Every problem meets the routine the batched tiers give a problem of its size.
__device__ inline void solve_r1_body_wide(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a,
                                          int64_t blk, int64_t nblk) {
    __shared__ double s_A[2 * 64 * 65];   // one matrix per wave
    __shared__ double s_x[3][128];
    __shared__ double s_z[128];
    extern __shared__ double s_tabr[];
    const int64_t count = *a.in_count;
    if (blk * 8 >= count) {
        write_block_stats(a.stat_rec + (int64_t)a.stat_off * 5, blk, ULLONG_MAX, 0, 0, 0, 0);
        return;
    }
    stage_to_lds(s_tabr, kt.Qs, (kt.qQ + 1) * TAY_NC);
    __syncthreads();
    const double* tQ = s_tabr;
    const int wave = threadIdx.x >> 6, lane16 = threadIdx.x & 15, grp = (threadIdx.x & 63) >> 4;
    const int gbase = (threadIdx.x & 63) - lane16;
    double* Ag = s_A + wave * 64 * 65;
    double* Ai = Ag + (threadIdx.x & 63) * 65;
    GroupStats st;
    for (int64_t base = (blk * 2 + wave) * 4; base < count; base += nblk * 8) {
        const int64_t qi = base + grp;
        const int l = qi < count ? glb(a.in_list)[qi] : -1;
        int n = 0;
        if (l >= 0) {
            int p1[1];
            gather_1d_rows<1>(g, nd, l, lane16, gbase, n, p1);
            if (n <= 32) r1_problem_ge<2>(g, nd, kt, a, l, tQ, st);
        }
        uint64_t wide = __ballot(l >= 0 && n > 32 && lane16 == 0);
        while (wide) {
            const int src = __ffsll((unsigned long long)wide) - 1;
            wide &= wide - 1ull;
            const int lw = __shfl(l, src, 64);
            r1_problem_lds<64>(g, nd, kt, a, lw, tQ, Ag, Ai, s_x, s_z, st);
        }
    }
    write_block_stats(a.stat_rec + (int64_t)a.stat_off * 5, blk, st.mn, st.mx, st.fail, st.empty, st.over);
}

template <int NL>
__global__ void __launch_bounds__(128, 2) k_solve_r1(Geo g, NodesDev nd, KTabDev kt, SolveArgs a) {
    clear_counters(a);
    if constexpr (NL == 64) solve_r1_body_wide(g, nd, kt, a, blockIdx.x, gridDim.x);
    else solve_r1_body<NL, true>(g, nd, kt, a, blockIdx.x, gridDim.x);
}

// A tier over the lists of all problems of a batch as one flat list: every workgroup reads the
// problems' list counts (FLAT_JOBS at a time) and their prefix sums, and each lane group takes one
// contiguous chunk of the concatenated lists (the problem of an entry by binary search).  A group's
// statistics go to each problem's one record of the tier with atomics, once per problem it visited;
// the records start neutral (k_batch_solve_reset).
constexpr int FLAT_JOBS = 1024;

template <int NL>
__global__ void __launch_bounds__(128, 2) k_solve_r1_flat(const SolveJob* __restrict__ jobs, int njobs) {
    constexpr int PER = FLAT_JOBS / 128;
    constexpr int GL = group_lanes<NL>();
    __shared__ double s_A[NL > 32 ? (128 / NL) * NL * (NL + 1) : 1];
    __shared__ double s_x[NL > 32 ? 3 : 1][128];
    __shared__ double s_z[NL > 32 ? 128 : 1];
    __shared__ int s_pre[FLAT_JOBS + 1];
    __shared__ int s_wsum[2];
    const int lane = threadIdx.x & (GL - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GL;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / GL;
    for (int j0 = 0; j0 < njobs; j0 += FLAT_JOBS) {
        const int nj = min(FLAT_JOBS, njobs - j0);
        // exclusive prefix sums of the counts, PER consecutive problems per thread
        int c[PER];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int jj = threadIdx.x * PER + k;
            c[k] = jj < nj ? glb(jobs[j0 + jj].a.in_count)[0] : 0;
            sum += c[k];
        }
        const int wl = threadIdx.x & 63, wv = threadIdx.x >> 6;
        int inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (wl >= o) inc += t;
        }
        if (wl == 63) s_wsum[wv] = inc;
        __syncthreads();
        int run = inc - sum + (wv ? s_wsum[0] : 0);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            s_pre[threadIdx.x * PER + k] = run;
            run += c[k];
        }
        if (threadIdx.x == 0) s_pre[FLAT_JOBS] = s_wsum[0] + s_wsum[1];
        __syncthreads();
        const int total = s_pre[nj];
        // contiguous chunks per group, so that a group's problems mostly share a job and its
        // statistics go out once per job (same-address atomics from every problem would serialise)
        const int64_t chunk = (total + ngroups - 1) / ngroups;
        const int64_t q0 = gid * chunk, q1 = min((int64_t)total, q0 + chunk);
        int cur = -1;
        GroupStats st;
        auto flush = [&]() {
            if (cur >= 0 && lane == 0) {
                const SolveJob& F = jobs[j0 + cur];
                unsigned long long* rec = (unsigned long long*)(F.a.stat_rec + (int64_t)F.a.stat_off * 5);
                if (st.mn != ULLONG_MAX) atomicMin(rec + 0, st.mn);
                if (st.mx) atomicMax(rec + 1, st.mx);
                if (st.fail) atomicAdd(rec + 2, st.fail);
                if (st.empty) atomicAdd(rec + 3, st.empty);
                if (st.over) atomicAdd(rec + 4, st.over);
            }
            st = GroupStats();
        };
        for (int64_t q = q0; q < q1; ++q) {
            // the last problem whose list starts at or before q (its count is then > 0)
            int lo = 0, hi = nj - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= q) lo = mid;
                else hi = mid - 1;
            }
            if (lo != cur) {
                flush();
                cur = lo;
            }
            const SolveJob& J = jobs[j0 + lo];
            const int l = glb(J.a.in_list)[q - s_pre[lo]];
            r1_solve<NL>(J.g, J.nd, J.kt, J.a, l, glb(J.kt.Qs), s_A, s_x, s_z, st);
        }
        flush();
        __syncthreads();   // s_pre and s_wsum are refilled for the next problems
    }
}

// ------------------------------------------------------------------ 1-D: one thread per problem
// For |I(l)| <= NMAX (the common case: about 2m members at one node per grid cell) a single thread
// holds the whole real system of the Sherman-Morrison form in registers: the lower triangle of A0,
// the three right-hand sides and the solution, with every loop unrolled.  Rows beyond n are padded
// with an identity block and zero right-hand sides, which decouples them exactly.
//
// A workgroup takes TPB consecutive grid indices.  Their members are consecutive sorted nodes
// p0(l) .. p0(l)+n-1, and (L_l^* L_l)[i][j] = M_sigma Qs(t_i - t_j) depends only on the node pair
// (t = M_sigma x = l0 + u), so every local matrix is a principal submatrix of one banded matrix
// over the workgroup's node range; the band (offsets 0 .. NMAX-1) is evaluated once in LDS.  The
// phase w_i = e^{i pi z_i / sigma} factors into e^{i pi l / sigma} e^{-i pi t_p / sigma}, the second
// factor per node.  Windows that wrap around the torus (the first 2m-1 grid indices) evaluate their
// entries directly.  Problems with more members or with a member on the window edge (tap 2m
// inside the support) are appended to the list of the group kernels.
constexpr int T1_TPB = T1_CELLS;

// 1 / sqrt(x) for x > 0: the hardware estimate and two Newton steps r <- r + r (1 - x r^2) / 2,
// each of which squares the relative error (to within a few units in the last place).
__device__ inline double rsqrt_refined(double x) {
    double r = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * r, r, 1.0);
        r = fma(0.5 * r, e, r);
    }
    return r;
}
// Appends l to list for every lane with f set: one atomic on the counter per wave, each lane's slot
// from its rank among the wave's flagged lanes.  Called by whole waves.
__device__ inline void append_wave(int* list, int* count, bool f, int l) {
    const uint64_t m = __ballot(f);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader, 64);
    if (f) glb(list)[base + __popcll(m & ((1ull << lane) - 1ull))] = l;
}
constexpr int T1_NODECAP = 448;   // staged nodes per workgroup (density up to ~1.7 per cell)

template <int NMAX>
__device__ inline void solve_t1_body(const Geo& g, const NodesDev& nd, const KTabDev& kt, const SolveArgs& a,
                                     int blk) {
    extern __shared__ double s_tabk[];                      // Ks Taylor table
    __shared__ double s_band[T1_NODECAP * NMAX];       // band of the workgroup's nodes, lambda on its diagonal
    // rows of the identity in the band's row addressing: entry (i, j) of row i at i + j (NMAX - 1)
    __shared__ double s_ident[NMAX * (NMAX - 1) + 1];
    __shared__ int s_l0[T1_NODECAP];                   // stencil base of the staged nodes
    __shared__ double s_u[T1_NODECAP];                 // offsets: t_p = l0_p + u_p
    __shared__ double2 s_phi[T1_NODECAP];              // e^{-i pi t_p / sigma}
    __shared__ int s_range[4];
    // Ks, read per member in the solves, is staged in LDS; Qs, read once per band entry, stays in
    // global memory (keeping LDS to four workgroups per CU)
    stage_to_lds(s_tabk, kt.Ks, (kt.qK + 1) * TAY_NC);

    const int Ms = g.Ms[0], w2 = 2 * g.m;
    const int L0 = blk * T1_TPB;
    const int l = L0 + threadIdx.x;
    // the first workgroup's windows wrap around the torus: it stages the nodes of the last 2m-1
    // cells first, with their stencil base shifted by -M_sigma, so that every window is one
    // contiguous range of the staged nodes (when the grid is long enough that the two parts differ)
    const bool circ = L0 == 0 && Ms > T1_TPB + w2;
    // node range of the workgroup: from the first member of problem L0 to the last of L0+TPB-1
    if (threadIdx.x == 0) {
        const int lo = max(L0 - w2 + 1, 0);
        const int hi = min(L0 + T1_TPB, Ms);
        s_range[0] = glb(nd.start)[lo];
        s_range[1] = glb(nd.start)[hi];
        s_range[2] = circ ? glb(nd.start)[Ms - w2 + 1] : 0;
        s_range[3] = circ ? glb(nd.start)[Ms] : 0;
    }
    __syncthreads();
    const int P0 = s_range[0];
    const int tS = s_range[2], ntail = s_range[3] - s_range[2];
    const int total = ntail + (s_range[1] - P0);
    const int nnode = min(total, T1_NODECAP);
    const bool staged = total <= T1_NODECAP;
    for (int i = threadIdx.x; i < nnode; i += blockDim.x) {
        const bool tail = i < ntail;
        const int p = tail ? tS + i : P0 + (i - ntail);
        s_l0[i] = glb(nd.l0s)[p] - (tail ? Ms : 0);
        s_u[i] = glb(nd.us)[p];
        // e^{-i pi t / sigma}, the integer part reduced exactly modulo 2 M_sigma
        const int64_t lm = ((int64_t)glb(nd.l0s)[p] * g.M[0]) % (2 * (int64_t)Ms);
        double sn, cs;
        sincospi((double)lm / (double)Ms + glb(nd.us)[p] * kt.inv_sigma, &sn, &cs);
        s_phi[i] = make_double2(cs, -sn);
    }
    __syncthreads();
    // offset-major order: the lanes of a wave take one offset d and consecutive nodes i, whose
    // arguments t_{i+d} - t_i lie close together, so a wave's table loads touch few cache lines
    // (node order would send each lane to a different part of the table)
    const uint32_t mg = (uint32_t)(0xFFFFFFFFu / (uint32_t)max(nnode, 1)) + 1u;   // e / nnode = e mg >> 32
    for (int e = threadIdx.x; e < nnode * NMAX; e += blockDim.x) {
        const int d = (int)__umulhi((uint32_t)e, mg), i = e - d * nnode;
        double v = 0.0;
        // t_{i+d} - t_i with the integer parts subtracted exactly
        if (i + d < nnode)
            v = kt.scaleG * tay_eval_r(glb(kt.Qs), kt.qQ, (double)(s_l0[i + d] - s_l0[i]) + (s_u[i + d] - s_u[i]));
        if (d == 0) v += kt.lam;
        s_band[i * NMAX + d] = v;
    }
    for (int k = threadIdx.x; k <= NMAX * (NMAX - 1); k += blockDim.x) s_ident[k] = (k % NMAX == 0) ? 1.0 : 0.0;
    __syncthreads();

    const double c1 = (double)Ms * kt.dM * kt.dM;
    unsigned long long st_min = ULLONG_MAX, st_max = 0, st_fail = 0, st_empty = 0, st_over = 0;
    int push_l = 0;   // 1: to a.out_list, 2: to a.out_list2
    if (l < Ms) {
        // members: cells l-2m+1 .. l, one range, or two when the window wraps (l < 2m-1)
        const int clo = l - w2 + 1;
        const bool wrap = clo < 0;
        int s0, n0, s1 = 0, n1 = 0;
        if (!wrap) {
            s0 = glb(nd.start)[clo];
            n0 = glb(nd.start)[l + 1] - s0;
        } else {
            s0 = glb(nd.start)[clo + Ms];
            n0 = glb(nd.start)[Ms] - s0;
            s1 = glb(nd.start)[0];
            n1 = glb(nd.start)[l + 1] - s1;
        }
        const int n = n0 + n1;
        // unstaged node ranges, oversized problems and (on short grids) windows that wrap around
        // the torus go to the group kernels
        bool fallback = (wrap && !circ) || n > NMAX || !staged;
        bool edge = false;
        {
            // the cell l-2m reaches l through its tap 2m only for nodes with u at m; the tap
            // 2m of every other node belongs to no problem and is zeroed here
            int ce = l - w2;
            if (ce < 0) ce += Ms;
            const int es = glb(nd.start)[ce], ee = glb(nd.start)[ce + 1];
            for (int p = es; p < ee; ++p) {
                if (edge_tap_member(glb(nd.us)[p], g.m)) {
                    edge = true;
                } else {
                    put_bopt(a.B64, a.B32, (int64_t)w2 * g.N + p, make_double2(0.0, 0.0));
                }
            }
        }
        if (fallback || edge) {
            // a batch sends a problem of 17 to 32 members whose count is exact (staged, no edge-tap
            // member, no wrap left to the group tiers) straight to its 32-member tier
            const bool wide = a.out_list2 && !edge && staged && !(wrap && !circ) && n > 16 && n <= 32;
            push_l = wide ? 2 : 1;
        } else if (n == 0) {
            ++st_empty;
        } else {
            st_min = n;
            st_max = n;
            const int b0 = wrap ? s0 - tS : ntail + (s0 - P0);   // first member in the staged range
            // e^{i pi l / sigma}, reduced exactly; w_i = e^{i pi (l - t_i) / sigma} from the staged
            // phases e^{-i pi t_i / sigma}
            double sl, cl;
            sincospi((double)(((int64_t)l * g.M[0]) % (2 * (int64_t)Ms)) / (double)Ms, &sl, &cl);
            // ---- A0 = M_sigma Qs(z_j - z_i) + lambda I from the band, Cholesky A0 = L L^T; the
            // diagonal keeps 1 / L[k][k].  Entry (i, j <= i) of the band lies at (b0 + j) NMAX + i - j,
            // so each row is read from one base address; rows past n read the identity instead.
            double A[NMAX * (NMAX + 1) / 2];
#pragma unroll
            for (int i = 0; i < NMAX; ++i) {
                const double* row = (i < n) ? s_band + b0 * NMAX + i : s_ident + i;
#pragma unroll
                for (int j = 0; j <= i; ++j) A[i * (i + 1) / 2 + j] = row[j * (NMAX - 1)];
            }
            bool ok = true;
#pragma unroll
            for (int k = 0; k < NMAX; ++k) {
                const double piv = A[k * (k + 1) / 2 + k];
                ok = ok && piv > 0.0;
                const double inv = rsqrt_refined(piv > 0.0 ? piv : 1.0);
                A[k * (k + 1) / 2 + k] = inv;
#pragma unroll
                for (int i = k + 1; i < NMAX; ++i) A[i * (i + 1) / 2 + k] *= inv;
#pragma unroll
                for (int i = k + 1; i < NMAX; ++i) {
                    const double lik = A[i * (i + 1) / 2 + k];
#pragma unroll
                    for (int j = k + 1; j <= i; ++j)
                        A[i * (i + 1) / 2 + j] = fma(-lik, A[j * (j + 1) / 2 + k], A[i * (i + 1) / 2 + j]);
                }
            }
            if (!ok) {
                ++st_fail;
            } else {
                // Sherman-Morrison through L alone: with y_w = L^{-1} w and y_k = L^{-1} Ks,
                //   s = w^* A0^{-1} w = |y_w|^2,   u^* Ks = w^* A0^{-1} Ks = y_w^* y_k,
                //   b = A0^{-1} (Ks + c' w) = L^{-T} (y_k + c' y_w),
                // so three right-hand sides go forward and two come back
                auto phase = [&](int i, double& wr, double& wi) {
                    const double2 ph = s_phi[b0 + i];
                    wr = cl * ph.x - sl * ph.y;
                    wi = cl * ph.y + sl * ph.x;
                };
                double xr[NMAX], xi[NMAX], xk[NMAX];
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    xr[i] = xi[i] = xk[i] = 0.0;
                    if (i < n) {
                        phase(i, xr[i], xi[i]);
                        xk[i] = tay_eval_r(s_tabk, kt.qK, (double)(l - s_l0[b0 + i]) - s_u[b0 + i]);
                    }
                }
                // forward: L y = x for the three right-hand sides
#pragma unroll
                for (int k = 0; k < NMAX; ++k) {
                    const double iv = A[k * (k + 1) / 2 + k];
                    xr[k] *= iv;
                    xi[k] *= iv;
                    xk[k] *= iv;
#pragma unroll
                    for (int i = k + 1; i < NMAX; ++i) {
                        const double lik = A[i * (i + 1) / 2 + k];
                        xr[i] = fma(-lik, xr[k], xr[i]);
                        xi[i] = fma(-lik, xi[k], xi[i]);
                        xk[i] = fma(-lik, xk[k], xk[i]);
                    }
                }
                double sdot = 0.0, wtr = 0.0, wti = 0.0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    sdot = fma(xr[i], xr[i], fma(xi[i], xi[i], sdot));
                    wtr = fma(xr[i], xk[i], wtr);
                    wti = fma(-xi[i], xk[i], wti);
                }
                const double den = 1.0 + c1 * sdot;
                const double cr = (kt.dM - c1 * wtr) / den, ci = (-c1 * wti) / den;
                // z = y_k + c' y_w, then back: L^T b = z (rows past n stay zero)
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const double zr = xk[i] + cr * xr[i] - ci * xi[i];
                    const double zi = cr * xi[i] + ci * xr[i];
                    xr[i] = zr;
                    xi[i] = zi;
                }
#pragma unroll
                for (int k = NMAX - 1; k >= 0; --k) {
                    const double iv = A[k * (k + 1) / 2 + k];
                    xr[k] *= iv;
                    xi[k] *= iv;
#pragma unroll
                    for (int i = 0; i < k; ++i) {
                        const double lki = A[k * (k + 1) / 2 + i];
                        xr[i] = fma(-lki, xr[k], xr[i]);
                        xi[i] = fma(-lki, xi[k], xi[i]);
                    }
                }
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    if (i < n) {
                        const double2 bb = make_double2(xr[i], xi[i]);
                        const int p = i < n0 ? s0 + i : s1 + (i - n0);   // sorted position
                        const int64_t idx = (int64_t)(l - s_l0[b0 + i]) * g.N + p;
                        put_bopt(a.B64, a.B32, idx, bb);
                    }
                }
            }
        }
    }
    // problems for the group tiers, appended with one atomic per wave and list (a list's counter is
    // shared by every workgroup of the problem: one atomic per lane would serialise on it)
    append_wave(a.out_list, a.out_count, push_l == 1, l);
    if (a.out_list2) append_wave(a.out_list2, a.out_count2, push_l == 2, l);
    write_block_stats(a.stat_rec + (int64_t)a.stat_off * 5, blk, st_min, st_max, st_fail, st_empty, st_over);
}

template <int NMAX>
__global__ void __launch_bounds__(T1_TPB, 2) k_solve_t1(Geo g, NodesDev nd, KTabDev kt, SolveArgs a) {
    reset_rec0(a);
    clear_counters(a);
    solve_t1_body<NMAX>(g, nd, kt, a, blockIdx.x);
}

template <int NMAX>
__global__ void __launch_bounds__(T1_TPB, 2) k_solve_t1_batched(const SolveJob* __restrict__ jobs,
                                                             const int2* __restrict__ bmap) {
    const int2 b = bmap[blockIdx.x];
    // the job by value: its fields then live in scalar registers (through a reference into
    // global memory they are reloaded around every store, which costs scratch)
    const SolveJob J = jobs[b.x];
    solve_t1_body<NMAX>(J.g, J.nd, J.kt, J.a, b.y);
}

void launch_solve_t1_batched(const SolveJob* jobs, const int2* t1_map, int t1_blocks, int qQ, int qK,
                             hipStream_t s) {
    const size_t shm = (size_t)(qK + 1) * TAY_NC * sizeof(double);
    if (t1_blocks > 0)
        hipLaunchKernelGGL((k_solve_t1_batched<13>), dim3(t1_blocks), dim3(T1_TPB), shm, s, jobs, t1_map);
}

// Per problem of a batch: reset the solver's status words (the node word stays), the four list
// counters (jobs of the thread tier, whose out_count is the first counter) and the one statistics
// record of each of the three list tiers (from the 16-lane tier's record on) to neutral.
__global__ void k_batch_solve_reset(const SolveJob* __restrict__ jobs, const SolveJob* __restrict__ tier_jobs,
                                    int njobs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    long long* st = jobs[j].a.status;
    for (int w = 0; w < STATUS_WORDS; ++w)
        if (w != ST_NONFINITE) st[w] = (w == ST_MIN_N) ? LLONG_MAX : 0;
    int* c = jobs[j].a.out_count;
    for (int i = 0; i < 4; ++i) c[i] = 0;
    long long* rec = tier_jobs[j].a.stat_rec + (int64_t)tier_jobs[j].a.stat_off * 5;
    for (int i = 0; i < 3 * 5; ++i) rec[i] = (i % 5 == 0) ? -1LL : 0;   // min as unsigned: ULLONG_MAX
}

// out[j] = the count of the list the job's tier wrote.
__global__ void k_batch_counts(const SolveJob* __restrict__ jobs, int njobs, int* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs) out[j] = *jobs[j].a.out_count;
}

void launch_batch_solve_reset(const SolveJob* jobs, int njobs, hipStream_t s) {
    if (njobs > 0)
        hipLaunchKernelGGL(k_batch_solve_reset, dim3((njobs + 255) / 256), dim3(256), 0, s, jobs, jobs + njobs, njobs);
}

void launch_batch_counts(const SolveJob* jobs, int njobs, int* out, hipStream_t s) {
    if (njobs > 0) hipLaunchKernelGGL(k_batch_counts, dim3((njobs + 255) / 256), dim3(256), 0, s, jobs, njobs, out);
}

void launch_solve_tier_batched(const SolveJob* jobs, int njobs, int nl, int blocks, hipStream_t s) {
    if (njobs <= 0 || blocks <= 0) return;
    if (nl == 16) hipLaunchKernelGGL((k_solve_r1_flat<16>), dim3(blocks), dim3(128), 0, s, jobs, njobs);
    else if (nl == 32) hipLaunchKernelGGL((k_solve_r1_flat<32>), dim3(blocks), dim3(128), 0, s, jobs, njobs);
    else hipLaunchKernelGGL((k_solve_r1_flat<64>), dim3(blocks), dim3(128), 0, s, jobs, njobs);
}

int launch_solve_thread_1d(const Geo& g, NodesDev nd, KTabDev kt, SolveArgs a, hipStream_t s) {
    const size_t shm = (size_t)(kt.qK + 1) * TAY_NC * sizeof(double);
    const unsigned blocks = (unsigned)((g.Ms[0] + T1_TPB - 1) / T1_TPB);
    hipLaunchKernelGGL((k_solve_t1<13>), dim3(blocks), dim3(T1_TPB), shm, s, g, nd, kt, a);
    return (int)blocks;
}


int launch_solve_tier(const Geo& g, NodesDev nd, KTabDev kt, SolveArgs a, int nl, hipStream_t s) {
    if (g.d == 1) {
        // Q table of at most (2*8*TAY_S+2)*TAY_NC doubles (about 21 KB) in LDS
        const size_t shm = (size_t)(kt.qQ + 1) * TAY_NC * sizeof(double);
        a.tables_in_lds = 1;
        int64_t b1 = (g.G + (128 / nl) - 1) / (128 / nl);
        // A list tier's problems are counted on the device, so its grid is sized for the longest
        // list; workgroups past the list exit at once.  Their registers (16-lane tier: two waves
        // per SIMD) and LDS (wide tier: the Q table and two 64 x 65 matrices, about 88 KB) bound how
        // many are resident per CU, so the cap is one dispatch round of 256 CUs: 4 and 1 per CU.
        const int64_t cap1 = !a.in_list ? 4096 : nl == 16 ? 1024 : 256;
        if (b1 > cap1) b1 = cap1;
        if (nl == 16) hipLaunchKernelGGL((k_solve_r1<16>), dim3((unsigned)b1), dim3(128), shm, s, g, nd, kt, a);
        else hipLaunchKernelGGL((k_solve_r1<64>), dim3((unsigned)b1), dim3(128), shm, s, g, nd, kt, a);
        return (int)b1;
    }
    const int64_t groups_per_block = 256 / nl;
    int64_t blocks = (g.G + groups_per_block - 1) / groups_per_block;
    const int64_t cap = a.in_list ? 512 : 2048;
    if (blocks > cap) blocks = cap;
    a.tables_in_lds = 0;
    if (nl == 16) hipLaunchKernelGGL((k_solve<2, 16>), dim3((unsigned)blocks), dim3(256), 0, s, g, nd, kt, a);
    else hipLaunchKernelGGL((k_solve<2, 32>), dim3((unsigned)blocks), dim3(256), 0, s, g, nd, kt, a);
    return (int)blocks;
}

}  // namespace infft
