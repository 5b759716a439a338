// Gradient of a real loss with respect to the node positions through B_opt(x) (implicit
// differentiation of the local problems of Algorithm 3.17).
//
// For fcheck = D^* F^* B_opt(x)^* f (3.32) with upstream gradient gfc (PyTorch's convention), the
// grid gradient is gdot = F D gfc and, per grid index l with members I(l),
//     bdot_j = sum_r conj(gdot_{r,l}) f_{r,j}          (gradient with respect to conj(b_j))
//     (G + lambda I) a = bdot                          (G Hermitian, the matrix of the solve)
//     dL = Re a^* (dr - dG b),
// since (G + lambda I) b = r.  Entry k of r = conj K(l/M_sigma - x) and row and column k of
// G[i][j] = M_sigma^d Q(x_i - x_j) move with x_k; membership is piecewise constant and has no
// derivative.  In grid units z = tau - u (so x_i - x_j = (z_j - z_i)/M_sigma) the contribution of
// problem l to dL/dx_{k,t} is
//     Re[ conj(a_k) (-M_t conj dK_t(z_k)) - conj(a_k) S M_t sum_j dQ_t(z_j - z_k) b_j
//         + b_k S M_t sum_i conj(a_i) dQ_t(z_k - z_i) ],        M_t = M_sigma,t, S = prod M_sigma,
// with dF_t the partial derivative in grid units along dimension t, from the Taylor tables.
// Layout of the work as in the solve tiers: a group of NL lanes per grid index, lane i owns
// member i and row i; problems with more members go to the next tier.
#include "internal.hpp"

namespace infft {

// F(z) and dF/dz from a Taylor table holding z >= 0 (F(-z) = conj F(z), so dF(-z) = -conj dF(z)).
__device__ inline void tay_eval_d(const double2* __restrict__ tab, int qmax, double z, double2& F,
                                  double2& dF) {
    const double az = fabs(z);
    int q = (int)rint(az * (double)TAY_S);
    if (q > qmax) q = qmax;
    const double e = az - (double)q * (1.0 / TAY_S);
    const double2* c = tab + (int64_t)q * TAY_NC;
    double2 acc = c[TAY_NC - 1], dacc = make_double2(0.0, 0.0);
#pragma unroll
    for (int p = TAY_NC - 2; p >= 0; --p) {
        dacc.x = fma(dacc.x, e, acc.x);
        dacc.y = fma(dacc.y, e, acc.y);
        const double2 cp = c[p];
        acc.x = fma(acc.x, e, cp.x);
        acc.y = fma(acc.y, e, cp.y);
    }
    if (z < 0.0) {
        F = make_double2(acc.x, -acc.y);
        dF = make_double2(-dacc.x, dacc.y);
    } else {
        F = acc;
        dF = dacc;
    }
}

// Partial derivative along dimension t of a tensor-product kernel at w (grid units).
template <int D>
__device__ inline double2 dkernel(const double2* const* tab, int qmax, double2 w, int t) {
    double2 F0, dF0;
    tay_eval_d(tab[0], qmax, w.x, F0, dF0);
    if (D == 1) return dF0;
    double2 F1, dF1;
    tay_eval_d(tab[1], qmax, w.y, F1, dF1);
    return t == 0 ? cmul(dF0, F1) : cmul(F0, dF1);
}

// QL: the Q Taylor table (1-D) is staged in LDS first; every lane evaluates it about 3n times per
// problem (its row of G, and dQ against each member), and from global memory each evaluation
// waited on ten dependent coefficient loads.
template <typename R, int D, int NL, bool QL>
__global__ void __launch_bounds__(256) k_bopt_grad(Geo g, NodesDev nd, KTabDev kt, BoptGradArgs ga) {
    using C = cx<R>;
    __shared__ double2 s_col[256];
    __shared__ double2 s_z[256];
    __shared__ double2 s_a[256];
    __shared__ double2 s_b[256];
    extern __shared__ double2 s_qtab[];
    const double2* qtab[MAX_D] = {kt.Q[0], kt.Q[1]};
    if (QL) {
        const int nq = (kt.qQ + 1) * TAY_NC;
        for (int i0 = threadIdx.x; i0 < nq; i0 += 8 * blockDim.x) {
            double2 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = i0 + k * blockDim.x;
                v[k] = kt.Q[0][min(i, nq - 1)];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = i0 + k * blockDim.x;
                if (i < nq) s_qtab[i] = v[k];
            }
        }
        __syncthreads();
        qtab[0] = s_qtab;
    }
    const int lane = threadIdx.x & (NL - 1);
    const int sb = threadIdx.x - lane;
    const int gbase = (threadIdx.x & 63) - lane;
    const uint64_t gmask = (NL == 64) ? ~0ull : ((1ull << NL) - 1ull);
    const int64_t gid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / NL;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / NL;
    const int64_t count = ga.in_list ? (int64_t)(*ga.in_count) : g.G;
    const int W = 2 * g.m + 1;
    const C* grid = (const C*)ga.grid;
    const C* f = (const C*)ga.f;

    for (int64_t qi = gid; qi < count; qi += ngroups) {
        const int l = ga.in_list ? ga.in_list[qi] : (int)qi;
        int n = 0, my_p = 0;
        if (D == 1) gather_1d(g, nd, l, lane, NL, gbase, gmask, n, my_p);
        else gather_2d(g, nd, l, lane, NL, gbase, gmask, n, my_p);
        if (n == 0) continue;
        if (n > NL) {
            if (lane == 0) {
                const int slot = atomicAdd(ga.out_count, 1);
                ga.out_list[slot] = l;
            }
            continue;
        }
        const bool act = lane < n;
        double z0 = 0.0, z1 = 0.0;
        double2 bval = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
        int my_j = 0;
        if (act) {
            int tap;
            if (D == 1) {
                int tau0 = l - nd.l0s[my_p];
                if (tau0 < 0) tau0 += g.Ms[0];
                z0 = (double)tau0 - nd.us[my_p];
                tap = tau0;
            } else {
                const int lc0 = l / g.Ms[1], lc1 = l - lc0 * g.Ms[1];
                int tau0 = lc0 - nd.l0s[(int64_t)my_p * 2];
                if (tau0 < 0) tau0 += g.Ms[0];
                int tau1 = lc1 - nd.l0s[(int64_t)my_p * 2 + 1];
                if (tau1 < 0) tau1 += g.Ms[1];
                z0 = (double)tau0 - nd.us[(int64_t)my_p * 2];
                z1 = (double)tau1 - nd.us[(int64_t)my_p * 2 + 1];
                tap = tau0 * W + tau1;
            }
            bval = ga.B64[(int64_t)tap * g.N + my_p];
            my_j = nd.perm[my_p];
            for (int r = 0; r < ga.nrhs; ++r) {
                const C gv = grid[(int64_t)r * g.G + l];
                const C fv = f[(int64_t)r * g.N + my_j];
                // conj(gv) * fv
                y.x += (double)gv.x * (double)fv.x + (double)gv.y * (double)fv.y;
                y.y += (double)gv.x * (double)fv.y - (double)gv.y * (double)fv.x;
            }
        }
        s_z[threadIdx.x] = make_double2(z0, z1);
        wave_sync();

        // ---- row i of G + lambda I
        double2 A[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            A[j] = make_double2(0.0, 0.0);
            if (j < n) {
                const double2 zj = s_z[sb + j];
                double2 qv = tay_eval(qtab[0], kt.qQ, zj.x - z0);
                if (D == 2) qv = cmul(qv, tay_eval(qtab[1], kt.qQ, zj.y - z1));
                A[j] = cscale(qv, kt.scaleG);
                if (j == lane) A[j] = make_double2(A[j].x + kt.lam, 0.0);
            }
        }
        // ---- Cholesky, lane i keeps row i of L (as in the solve tiers) and 1 / L[i][i]
        bool ok = true;
        double dinv = 1.0;
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
                if (lane == k) {
                    A[k] = make_double2(sq, 0.0);
                    dinv = inv;
                } else if (lane > k) {
                    A[k] = cscale(A[k], inv);
                }
                wave_sync();
            }
        }
        if (!ok) continue;   // counted by the precompute; its column of B_opt is zero
        // ---- a = (L L^*)^{-1} bdot
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (k < n) {
                if (lane == k) y = cscale(y, dinv);
                s_col[threadIdx.x] = y;
                wave_sync();
                const double2 yk = s_col[sb + k];
                if (lane > k && act) y = csub(y, cmul(A[k], yk));
                wave_sync();
            }
        }
        double2 a = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = NL - 1; k >= 0; --k) {
            if (k < n) {
                s_col[threadIdx.x] = (lane > k && act) ? cmul(cconj(A[k]), a) : make_double2(0.0, 0.0);
                wave_sync();
                if (lane == k) {
                    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
                    for (int j = k + 1; j < NL; ++j) sum = cadd(sum, s_col[sb + j]);
                    a = cscale(csub(y, sum), dinv);
                }
                wave_sync();
            }
        }
        s_a[threadIdx.x] = act ? a : make_double2(0.0, 0.0);
        s_b[threadIdx.x] = bval;
        wave_sync();
        // ---- the node gradient of member lane
        if (act) {
            const double2 zk = make_double2(z0, z1);
            for (int t = 0; t < D; ++t) {
                const double Mt = (double)g.Ms[t];
                const double2 dK = dkernel<D>(kt.K, kt.qK, zk, t);
                double2 srow = make_double2(0.0, 0.0), scol = make_double2(0.0, 0.0);
                for (int j = 0; j < n; ++j) {
                    const double2 zj = s_z[sb + j];
                    // dQ_t(-w) = -conj dQ_t(w) (the tables hold w >= 0 and the sign is applied after
                    // the evaluation, so this is exact for w != 0; at w = 0, j = k, the real part
                    // of dQ_t(0) is zero up to rounding)
                    const double2 dq_row = dkernel<D>(qtab, kt.qQ, make_double2(zj.x - zk.x, zj.y - zk.y), t);
                    const double2 dq_col = make_double2(-dq_row.x, dq_row.y);
                    srow = cadd(srow, cmul(dq_row, s_b[sb + j]));
                    scol = cadd(scol, cmul(cconj(s_a[sb + j]), dq_col));
                }
                const double2 ca = cconj(a);
                const double2 dr = make_double2(-Mt * dK.x, Mt * dK.y);   // -conj(M_t dK)
                const double2 v = cadd(csub(cmul(ca, dr), cscale(cmul(ca, srow), kt.scaleG * Mt)),
                                       cscale(cmul(bval, scol), kt.scaleG * Mt));
                atomicAdd(&ga.gradx[(int64_t)my_j * D + t], v.x);
            }
        }
        wave_sync();
    }
}

template <typename R>
int launch_bopt_grad(const Geo& g, NodesDev nd, KTabDev kt, BoptGradArgs ga, int nl, hipStream_t s) {
    const int64_t groups_per_block = 256 / nl;
    int64_t blocks = (g.G + groups_per_block - 1) / groups_per_block;
    // 1-D: the Q table in LDS when it fits beside the 16 KB of the kernel's own arrays within
    // 64 KB (m <= 9); then two workgroups per CU, each staging it once for many problems
    const size_t qbytes = (size_t)(kt.qQ + 1) * TAY_NC * sizeof(double2);
    const bool ql = g.d == 1 && qbytes <= 48 * 1024;
    const int64_t cap = ql ? 512 : ga.in_list ? 512 : 2048;
    if (blocks > cap) blocks = cap;
#define INFFT_BG(D_, NL_, QL_)                                                                              \
    hipLaunchKernelGGL((k_bopt_grad<R, D_, NL_, QL_>), dim3((unsigned)blocks), dim3(256), QL_ ? qbytes : 0, s, \
                       g, nd, kt, ga)
    if (g.d == 1) {
        if (ql) {
            if (nl == 16) INFFT_BG(1, 16, true);
            else INFFT_BG(1, 32, true);
        } else {
            if (nl == 16) INFFT_BG(1, 16, false);
            else INFFT_BG(1, 32, false);
        }
    } else {
        if (nl == 16) INFFT_BG(2, 16, false);
        else INFFT_BG(2, 32, false);
    }
#undef INFFT_BG
    return (int)blocks;
}

template int launch_bopt_grad<float>(const Geo&, NodesDev, KTabDev, BoptGradArgs, int, hipStream_t);
template int launch_bopt_grad<double>(const Geo&, NodesDev, KTabDev, BoptGradArgs, int, hipStream_t);

// One workgroup per large problem of a batch, after the blocked factorisation: bdot from the
// grid gradient and the samples, a = (L L^*)^{-1} bdot, then the member gradients (members in
// the workgroup's threads, the sums over the other members in a loop).
template <typename R, int D>
__global__ void __launch_bounds__(BIG_TPB) k_big_grad(Geo g, BigArgs a, KTabDev kt, BoptGradArgs ga,
                                                      const int* __restrict__ perm) {
    using C = cx<R>;
    if (a.stale && *a.stale) return;
    const BigProb P = a.probs[blockIdx.x];
    if (a.fail[P.id]) return;   // uniform: a failed problem has no usable factor
    const double2* A = a.A + P.off;
    double2* y = a.mr + P.moff;
    double2* bv = a.mb + P.moff;
    const double2* z = a.mz + P.moff;
    const int* midx = a.midx + P.moff;
    const int* mtap = a.mtap + P.moff;
    const C* grid = (const C*)ga.grid;
    const C* f = (const C*)ga.f;
    for (int i = threadIdx.x; i < P.n; i += BIG_TPB) {
        const int p = midx[i];
        const int j = perm[p];
        double2 s = make_double2(0.0, 0.0);
        for (int r = 0; r < ga.nrhs; ++r) {
            const C gv = grid[(int64_t)r * g.G + P.l];
            const C fv = f[(int64_t)r * g.N + j];
            s.x += (double)gv.x * (double)fv.x + (double)gv.y * (double)fv.y;
            s.y += (double)gv.x * (double)fv.y - (double)gv.y * (double)fv.x;
        }
        y[i] = s;
        bv[i] = ga.B64[(int64_t)mtap[i] * g.N + p];
    }
    __syncthreads();
    big_substitute(P, A, y, P.nblk);
    __syncthreads();
    for (int k = threadIdx.x; k < P.n; k += BIG_TPB) {
        const double2 zk = z[k], ak = y[k], bk = bv[k];
        const int jk = perm[midx[k]];
        for (int t = 0; t < D; ++t) {
            const double Mt = (double)g.Ms[t];
            const double2 dK = dkernel<D>(kt.K, kt.qK, zk, t);
            double2 srow = make_double2(0.0, 0.0), scol = make_double2(0.0, 0.0);
            for (int j = 0; j < P.n; ++j) {
                const double2 zj = z[j];
                const double2 dq_row = dkernel<D>(kt.Q, kt.qQ, make_double2(zj.x - zk.x, zj.y - zk.y), t);
                const double2 dq_col = dkernel<D>(kt.Q, kt.qQ, make_double2(zk.x - zj.x, zk.y - zj.y), t);
                srow = cadd(srow, cmul(dq_row, bv[j]));
                scol = cadd(scol, cmul(cconj(y[j]), dq_col));
            }
            const double2 ca = cconj(ak);
            const double2 dr = make_double2(-Mt * dK.x, Mt * dK.y);
            const double2 v = cadd(csub(cmul(ca, dr), cscale(cmul(ca, srow), kt.scaleG * Mt)),
                                   cscale(cmul(bk, scol), kt.scaleG * Mt));
            atomicAdd(&ga.gradx[(int64_t)jk * D + t], v.x);
        }
    }
}

void launch_big_grad(const Geo& g, BigArgs a, KTabDev kt, BoptGradArgs ga, const int* perm, int nprob, bool f32,
                     hipStream_t s) {
    if (nprob <= 0) return;
    const dim3 gr(nprob), bl(BIG_TPB);
    if (g.d == 1) {
        if (f32) hipLaunchKernelGGL((k_big_grad<float, 1>), gr, bl, 0, s, g, a, kt, ga, perm);
        else hipLaunchKernelGGL((k_big_grad<double, 1>), gr, bl, 0, s, g, a, kt, ga, perm);
    } else {
        if (f32) hipLaunchKernelGGL((k_big_grad<float, 2>), gr, bl, 0, s, g, a, kt, ga, perm);
        else hipLaunchKernelGGL((k_big_grad<double, 2>), gr, bl, 0, s, g, a, kt, ga, perm);
    }
}

}  // namespace infft
