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
// Layout of the work: a group of NL lanes (NL = 16 or 32) owns one grid index at a time.  The
// members of I(l) are gathered from the (2m+1)^d grid cells whose nodes reach l (the node CSR);
// lane i owns member i and row i of the Hermitian system.  The Cholesky factorisation, forward
// and backward substitution run across the group with register rows and cross-lane shuffles.
// Problems with more than NL members are passed on to the next, wider group size.
#include "internal.hpp"

#include <limits.h>

namespace infft {

__device__ inline double2 tay_eval(const double2* __restrict__ tab, int qmax, double z) {
    const double az = fabs(z);
    int q = (int)rint(az * (double)TAY_S);
    if (q > qmax) q = qmax;
    const double e = az - (double)q * (1.0 / TAY_S);
    const double2* c = tab + (int64_t)q * TAY_NC;
    double2 acc = c[TAY_NC - 1];
#pragma unroll
    for (int p = TAY_NC - 2; p >= 0; --p) {
        const double2 cp = c[p];
        acc.x = fma(acc.x, e, cp.x);
        acc.y = fma(acc.y, e, cp.y);
    }
    if (z < 0.0) acc.y = -acc.y;
    return acc;
}

__device__ inline double2 shfl2(double2 v, int src) {
    return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

template <int D, int NL>
__global__ void __launch_bounds__(256) k_solve(Geo g, NodesDev nd, KTabDev kt, SolveArgs a) {
    const int lane = threadIdx.x & (NL - 1);
    const int gbase = (threadIdx.x & 63) - lane;
    const uint64_t gmask = (NL == 64) ? ~0ull : ((1ull << NL) - 1ull);
    const int64_t gid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / NL;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / NL;
    const int64_t count = a.in_list ? (int64_t)(*a.in_count) : g.G;
    const int m = g.m, W = 2 * g.m + 1, w2 = 2 * g.m;
    const int ncell = (D == 2) ? W * W : W;

    unsigned long long st_min = ULLONG_MAX, st_max = 0, st_fail = 0, st_empty = 0, st_over = 0;

    for (int64_t qi = gid; qi < count; qi += ngroups) {
        const int l = a.in_list ? a.in_list[qi] : (int)qi;
        const int lc0 = (D == 2) ? l / g.Ms[1] : l;
        const int lc1 = (D == 2) ? l - lc0 * g.Ms[1] : 0;

        // ---- members of I(l): nodes of the cells l - tau, tau in {0..2m}^d
        int n = 0;
        int my_p = 0, my_tau = 0;
        for (int c = 0; c < ncell; ++c) {
            const int tau0 = (D == 2) ? c / W : c;
            const int tau1 = (D == 2) ? c - tau0 * W : 0;
            int c0 = lc0 - tau0;
            if (c0 < 0) c0 += g.Ms[0];
            int c1 = lc1 - tau1;
            if (c1 < 0) c1 += g.Ms[1];
            const int64_t key = cell_key(g, c0, c1);
            const int s = nd.start[key], e = nd.start[key + 1];
            if (s == e) continue;
            const bool edge = (tau0 == w2) || (D == 2 && tau1 == w2);
            if (!edge) {
                // tau < 2m in every dimension: |u - tau| <= m holds for every node of the cell
                const int k = lane - n;
                if (k >= 0 && k < e - s) {
                    my_p = s + k;
                    my_tau = c;
                }
                n += e - s;
            } else {
                // tau = 2m reaches l only when u = m exactly (node on a grid point)
                for (int base = s; base < e; base += NL) {
                    const int p = base + lane;
                    bool mem = p < e;
                    if (mem && tau0 == w2) mem = nd.us[(int64_t)p * D] == (double)m;
                    if (mem && D == 2 && tau1 == w2) mem = nd.us[(int64_t)p * D + 1] == (double)m;
                    const uint64_t gm = (__ballot(mem) >> gbase) & gmask;
                    const int cnt = __popcll(gm);
                    const int k = lane - n;
                    if (k >= 0 && k < cnt) {
                        uint64_t mm = gm;
                        for (int i = 0; i < k; ++i) mm &= mm - 1ull;
                        my_p = base + (__ffsll((unsigned long long)mm) - 1);
                        my_tau = c;
                    }
                    n += cnt;
                }
            }
        }
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

        // ---- z_i = tau_i - u_i per dimension; right-hand side r_i = conj K(z_i)
        double z0 = 0.0, z1 = 0.0;
        double2 y = make_double2(0.0, 0.0);
        if (act) {
            const int tau0 = (D == 2) ? my_tau / W : my_tau;
            z0 = (double)tau0 - nd.us[(int64_t)my_p * D];
            double2 kv = tay_eval(kt.K[0], kt.qK, z0);
            if (D == 2) {
                const int tau1 = my_tau - tau0 * W;
                z1 = (double)tau1 - nd.us[(int64_t)my_p * D + 1];
                kv = cmul(kv, tay_eval(kt.K[1], kt.qK, z1));
            }
            y = cconj(kv);
        }

        // ---- row i of G + lambda I (lower triangle): G[i][j] = M_sigma^d Q(z_j - z_i)
        double2 A[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const double zj0 = __shfl(z0, gbase + j, 64);
            const double zj1 = (D == 2) ? __shfl(z1, gbase + j, 64) : 0.0;
            A[j] = make_double2(0.0, 0.0);
            if (act && j < n && j <= lane) {
                double2 qv = tay_eval(kt.Q[0], kt.qQ, zj0 - z0);
                if (D == 2) qv = cmul(qv, tay_eval(kt.Q[1], kt.qQ, zj1 - z1));
                A[j] = cscale(qv, kt.scaleG);
                if (j == lane) A[j] = make_double2(A[j].x + kt.lam, 0.0);
            }
        }

        // ---- Cholesky G + lambda I = L L^*, lane i keeps row i of L
        bool ok = true;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (k < n && ok) {
                const double piv = __shfl(A[k].x, gbase + k, 64);
                if (!(piv > 0.0)) {
                    ok = false;
                } else {
                    const double sq = sqrt(piv), inv = 1.0 / sq;
                    if (lane == k) A[k] = make_double2(sq, 0.0);
                    else if (lane > k) A[k] = cscale(A[k], inv);
#pragma unroll
                    for (int j = k + 1; j < NL; ++j) {
                        if (j < n) {
                            const double2 Ljk = shfl2(A[k], gbase + j);
                            if (lane >= j && act) A[j] = csub(A[j], cmulc(A[k], Ljk));
                        }
                    }
                }
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
                const double Lkk = __shfl(A[k].x, gbase + k, 64);
                const double2 yk = cscale(shfl2(y, gbase + k), 1.0 / Lkk);
                if (lane == k) y = yk;
                else if (lane > k && act) y = csub(y, cmul(A[k], yk));
            }
        }
        // ---- backward substitution L^* b = y
        double2 bsol = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = NL - 1; k >= 0; --k) {
            if (k < n) {
                double2 c = make_double2(0.0, 0.0);
                if (lane > k && act) c = cmul(cconj(A[k]), bsol);
#pragma unroll
                for (int o = NL / 2; o >= 1; o >>= 1) {
                    c.x += __shfl_xor(c.x, o, 64);
                    c.y += __shfl_xor(c.y, o, 64);
                }
                const double Lkk = __shfl(A[k].x, gbase + k, 64);
                const double2 yk = shfl2(y, gbase + k);
                if (lane == k) bsol = cscale(csub(yk, c), 1.0 / Lkk);
            }
        }

        // ---- scatter into B_opt ([tap][sorted node])
        if (act) {
            const int64_t idx = (int64_t)my_tau * g.N + my_p;
            a.B64[idx] = bsol;
            if (a.B32) a.B32[idx] = make_float2((float)bsol.x, (float)bsol.y);
        }
    }

    // ---- statistics: reduce over the wave, one set of atomics per wave
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        st_min = min(st_min, (unsigned long long)__shfl_xor((long long)st_min, o, 64));
        st_max = max(st_max, (unsigned long long)__shfl_xor((long long)st_max, o, 64));
        st_fail += (unsigned long long)__shfl_xor((long long)st_fail, o, 64);
        st_empty += (unsigned long long)__shfl_xor((long long)st_empty, o, 64);
        st_over += (unsigned long long)__shfl_xor((long long)st_over, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        unsigned long long* st = (unsigned long long*)a.status;
        if (st_min != ULLONG_MAX) atomicMin(&st[ST_MIN_N], st_min);
        if (st_max) atomicMax(&st[ST_MAX_N], st_max);
        if (st_fail) atomicAdd(&st[ST_FAILED], st_fail);
        if (st_empty) atomicAdd(&st[ST_EMPTY], st_empty);
        if (st_over) atomicAdd(&st[ST_OVERSIZED], st_over);
    }
}

int solve_max_supported() { return 32; }

void launch_solve_tier(const Geo& g, NodesDev nd, KTabDev kt, SolveArgs a, int nl, hipStream_t s) {
    const int64_t groups_per_block = 256 / nl;
    int64_t blocks = (g.G + groups_per_block - 1) / groups_per_block;
    const int64_t cap = a.in_list ? 1024 : 8192;
    if (blocks > cap) blocks = cap;
    if (g.d == 1) {
        if (nl == 16) hipLaunchKernelGGL((k_solve<1, 16>), dim3((unsigned)blocks), dim3(256), 0, s, g, nd, kt, a);
        else hipLaunchKernelGGL((k_solve<1, 32>), dim3((unsigned)blocks), dim3(256), 0, s, g, nd, kt, a);
    } else {
        if (nl == 16) hipLaunchKernelGGL((k_solve<2, 16>), dim3((unsigned)blocks), dim3(256), 0, s, g, nd, kt, a);
        else hipLaunchKernelGGL((k_solve<2, 32>), dim3((unsigned)blocks), dim3(256), 0, s, g, nd, kt, a);
    }
}

}  // namespace infft
