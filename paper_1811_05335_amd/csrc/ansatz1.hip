// Ansatz 1 (Section 3.2.1, Algorithm 3.10): per-node optimisation of the columns of B^*.
//
// Node j solves min ||K_j y - e_j||^2 + lambda_j ||y||^2 over the members of I(x_j) (3.16), with
// K_j the columns l in I(x_j) of K = A D^* F^* (3.14), K[h, l] = K(x_h - l/M_sigma), and the
// normal equations (K_j^* K_j + lambda_j I) y = K_j^* e_j (3.22).  The Gram matrix of every node is
// a window of one banded table: (K^* K)[l, l+d] = S(l, d) depends only on the grid pair, and
// K^* K = F D (A^* A) D^* F^* with A^* A Toeplitz of symbol P(q) = sum_h e^{2 pi i q x_h}, so
//
//   S(l, d) = sum_{|q| < M} P(q) R_d(q) e^{-2 pi i q l / M_sigma},
//   R_d(q)  = sum_k D_k D_{k+q} e^{-2 pi i (k+q) d / M_sigma}.
//
// R_d comes from grid samples: with a[s] = K(s/M_sigma) = sum_k D_k e^{2 pi i k s / M_sigma},
// conj(a[s]) a[s - d] holds the frequencies q = k' - k, |q| < M, of R_d, so for M_sigma >= 2M - 1
// (sigma >= 2) its length-M_sigma DFT gives R_d without aliasing.  Below that the coefficient range
// is split into two half bands a^lo, a^hi: conj(a^b[s]) a^c[s - d] holds the frequencies with k in
// b and k' in c, a range of width < M <= M_sigma, so four such products cover every sigma >= 1.
// This replaces the
// paper's N NFFTs of length N(2m+1) (O(N^2)) by O(m M_sigma log M_sigma) FFT work and one
// adjoint NFFT of bandwidth 2M for P.
//
// All arithmetic here is FP64.  The host side (abi.cpp) runs the FFTs and the adjoint NFFT.

#include "internal.hpp"

namespace infft {
namespace {

// Band indicators as FFT inputs, [nb][M]: nb = 1 the whole range; nb = 2 the half bands, band 0
// k < 0 and band 1 k >= 0.
__global__ void k_a1_bands(double2* __restrict__ out, int M, int nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb * M) return;
    const int band = i / M, k = i - band * M;     // k is the centred index + M/2
    const bool on = nb == 1 || ((band == 0) ? (k < M / 2) : (k >= M / 2));
    out[i] = make_double2(on ? 1.0 : 0.0, 0.0);
}

// Frequency range of pair c: one pair (whole band) |q| < M; four pairs (lo,lo), (hi,hi), (lo,hi),
// (hi,lo).
__device__ inline void pair_range(int c, int npair, int M, int& lo, int& hi) {
    if (npair == 1) {
        lo = -(M - 1);
        hi = M - 1;
    } else {
        lo = c < 2 ? -(M / 2 - 1) : (c == 2 ? 1 : -(M - 1));
        hi = c < 2 ? (M / 2 - 1) : (c == 2 ? (M - 1) : -1);
    }
}

__global__ void k_a1_ones(double2* __restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_double2(1.0, 0.0);
}

// prod[c][dd][s] = conj(a^b[s]) a^b'[(s - d) mod M_sigma] * scale for the pairs c (one pair: the
// whole band; four: (lo,lo), (hi,hi), (lo,hi), (hi,lo)) and d = d0 + dd.
__global__ void k_a1_products(const double2* __restrict__ a, double2* __restrict__ prod, int Ms, int d0, int nd,
                              int npair, double scale) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)npair * nd * Ms;
    if (i >= total) return;
    const int s = (int)(i % Ms);
    const int64_t r = i / Ms;
    const int dd = (int)(r % nd);
    const int c = (int)(r / nd);
    const int bl = (c == 1 || c == 3) ? 1 : 0;   // band of k (always 0 for one pair)
    const int br = (c == 1 || c == 2) ? 1 : 0;   // band of k + q
    int sd = s - (d0 + dd);
    if (sd < 0) sd += Ms;
    const double2 u = a[(int64_t)bl * Ms + s];
    const double2 v = a[(int64_t)br * Ms + sd];
    prod[i] = make_double2((u.x * v.x + u.y * v.y) * scale, (u.x * v.y - u.y * v.x) * scale);
}

// V[dd][r] = sum_c P(q_c(r)) R_c[dd][r], q_c(r) the representative of r mod M_sigma inside pair c's
// frequency range; P(q) = h[M - q] with h the adjoint NFFT of ones at bandwidth 2M
// (h_k = sum_h e^{-2 pi i k x_h}, k = -M .. M-1).
__global__ void k_a1_fold(const double2* __restrict__ R, const double2* __restrict__ h, double2* __restrict__ V,
                          int M, int Ms, int nd, int npair) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nd * Ms) return;
    const int r = (int)(i % Ms);
    const int dd = (int)(i / Ms);
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < npair; ++c) {
        int lo, hi;
        pair_range(c, npair, M, lo, hi);
        const int q = r <= hi ? r : r - Ms;
        if (q < lo || q > hi) continue;
        const double2 p = h[M - q];
        const double2 v = R[((int64_t)c * nd + dd) * Ms + r];
        acc.x += p.x * v.x - p.y * v.y;
        acc.y += p.x * v.y + p.y * v.x;
    }
    V[i] = acc;
}

inline __device__ constexpr int tri(int a, int b) { return a * (a + 1) / 2 + b; }

// Matrix storage of the per-node solve: registers (small systems) or one LDS column per thread.
template <int NE, int TPB, bool REG>
struct SolveStore;
template <int NE, int TPB>
struct SolveStore<NE, TPB, true> {
    double2 v[NE];
    __device__ double2& operator()(int i, int) { return v[i]; }
};
template <int NE, int TPB>
struct SolveStore<NE, TPB, false> {
    double2 (*s)[TPB];
    __device__ double2& operator()(int i, int t) { return s[i][t]; }
};

// One thread per node (sorted order).  The Hermitian system over the 2m+1 taps keeps identity
// rows for taps outside I(x_j), so their entries come out zero; the packed lower triangle lives in
// registers for 2m+1 <= 9 and in LDS (one column per thread) above.  B_opt^* column j is stored as
// rows[tau][p] = conj(y_tau), which makes the modified adjoint D^* F^* B^* f equal
// (1/M) D^* F^* B_opt^* f of the paper.
template <int NT, int TPB, bool REG>
__global__ __launch_bounds__(TPB) void k_a1_solve(Geo g, NodesDev nd, const double2* __restrict__ S,
                                                  const double2* __restrict__ Ktab, int qK, double rho,
                                                  double2* __restrict__ B64, float2* __restrict__ Blo,
                                                  long long* __restrict__ status) {
    constexpr int NE = NT * (NT + 1) / 2;
    constexpr int LDS_NE = REG ? 1 : NE;
    constexpr int LDS_NT = REG ? 1 : NT;
    __shared__ double2 s_A[LDS_NE][TPB];
    __shared__ double2 s_y[LDS_NT][TPB];
    __shared__ unsigned long long s_mn, s_mx, s_fail;
    const int t = threadIdx.x;
    if (t == 0) {
        s_mn = ~0ull;
        s_mx = 0ull;
        s_fail = 0ull;
    }
    __syncthreads();
    SolveStore<NE, TPB, REG> A;
    SolveStore<NT, TPB, REG> y;
    if constexpr (!REG) {
        A.s = s_A;
        y.s = s_y;
    }
    constexpr int UNR = REG ? NT : 1;   // LDS storage: rolled loops keep the code and registers small
    const int64_t p = blockIdx.x * (int64_t)TPB + t;
    const int Ms = g.Ms[0], m = g.m;
    const int n = 2 * m + 1;
    if (p < g.N) {
        const int l0 = nd.l0s[p];
        const double u = nd.us[p];
        unsigned mem = 0u;   // bit a: tap a is in I(x_j)
        int cnt = 0;
        double tr = 0.0;
#pragma unroll UNR
        for (int a = 0; a < NT; ++a) {
            const bool in = a < n && isfinite(u) && (a < 2 * m || edge_tap_member(u, m));
            mem |= (in ? 1u : 0u) << a;
            double2 r = make_double2(0.0, 0.0);
            if (in) {
                ++cnt;
                int la = l0 + a;
                if (la >= Ms) la -= Ms;
                tr += S[la].x;
                // K_j^* e_j entry: conj K((u - tau)/M_sigma) = K((tau - u)/M_sigma)
                r = tay_eval(Ktab, qK, (double)a - u);
            }
            y(a, t) = r;
        }
        const double lam = cnt > 0 ? rho * tr / (double)cnt : 0.0;
        // Gram: entry (a, b), a >= b, is (K^* K)[l_a, l_b] = conj S(l_b, a - b)
#pragma unroll UNR
        for (int a = 0; a < NT; ++a) {
#pragma unroll UNR
            for (int b = 0; b <= a; ++b) {
                double2 v = make_double2(0.0, 0.0);
                if ((mem >> a) & (mem >> b) & 1u) {
                    int lb = l0 + b;
                    if (lb >= Ms) lb -= Ms;
                    const double2 sv = S[(int64_t)(a - b) * Ms + lb];
                    v = make_double2(sv.x, a == b ? 0.0 : -sv.y);
                    if (a == b) v.x += lam;
                } else if (a == b) {
                    v.x = 1.0;
                }
                A(tri(a, b), t) = v;
            }
        }
        // Cholesky A = L L^*; the reciprocal of each pivot replaces it on the diagonal.  A pivot
        // <= 0 marks the solve failed (the loop runs on with a unit pivot and the result is dropped).
        bool ok = cnt > 0;
#pragma unroll UNR
        for (int j = 0; j < NT; ++j) {
            double sd = A(tri(j, j), t).x;
#pragma unroll UNR
            for (int k = 0; k < j; ++k) {
                const double2 l = A(tri(j, k), t);
                sd -= l.x * l.x + l.y * l.y;
            }
            if (!(sd > 0.0)) {
                ok = false;
                sd = 1.0;
            }
            const double inv = 1.0 / sqrt(sd);
            A(tri(j, j), t) = make_double2(inv, 0.0);
#pragma unroll UNR
            for (int i = j + 1; i < NT; ++i) {
                double2 v = A(tri(i, j), t);
#pragma unroll UNR
                for (int k = 0; k < j; ++k) {
                    const double2 li = A(tri(i, k), t), lj = A(tri(j, k), t);
                    // v -= L[i][k] conj(L[j][k])
                    v.x -= li.x * lj.x + li.y * lj.y;
                    v.y -= li.y * lj.x - li.x * lj.y;
                }
                A(tri(i, j), t) = make_double2(v.x * inv, v.y * inv);
            }
        }
        // L z = r, then L^* y = z
#pragma unroll UNR
        for (int i = 0; i < NT; ++i) {
            double2 v = y(i, t);
#pragma unroll UNR
            for (int k = 0; k < i; ++k) {
                const double2 l = A(tri(i, k), t), yk = y(k, t);
                v.x -= l.x * yk.x - l.y * yk.y;
                v.y -= l.x * yk.y + l.y * yk.x;
            }
            const double inv = A(tri(i, i), t).x;
            y(i, t) = make_double2(v.x * inv, v.y * inv);
        }
#pragma unroll UNR
        for (int i = NT - 1; i >= 0; --i) {
            double2 v = y(i, t);
#pragma unroll UNR
            for (int k = i + 1; k < NT; ++k) {
                const double2 l = A(tri(k, i), t), yk = y(k, t);   // conj(L[k][i]) y_k
                v.x -= l.x * yk.x + l.y * yk.y;
                v.y -= l.x * yk.y - l.y * yk.x;
            }
            const double inv = A(tri(i, i), t).x;
            y(i, t) = make_double2(v.x * inv, v.y * inv);
        }
        if (!ok && cnt > 0) atomicAdd(&s_fail, 1ull);
#pragma unroll UNR
        for (int a = 0; a < NT; ++a) {
            if (a >= n) continue;
            const double2 ya = y(a, t);
            const double2 v = (ok && ((mem >> a) & 1u)) ? make_double2(ya.x, -ya.y) : make_double2(0.0, 0.0);
            B64[(int64_t)a * g.N + p] = v;
            if (Blo) Blo[(int64_t)a * g.N + p] = make_float2((float)v.x, (float)v.y);
        }
        if (cnt > 0) {
            atomicMin(&s_mn, (unsigned long long)cnt);
            atomicMax(&s_mx, (unsigned long long)cnt);
        }
    }
    __syncthreads();
    if (t == 0) {
        if (s_fail) atomicAdd((unsigned long long*)&status[ST_FAILED], s_fail);
        if (s_mx) {
            atomicMin((unsigned long long*)&status[ST_MIN_N], s_mn);
            atomicMax((unsigned long long*)&status[ST_MAX_N], s_mx);
        }
    }
}

template <int NT, int TPB, bool REG>
void a1_solve_launch(const Geo& g, const NodesDev& nd, const double2* S, const double2* Ktab, int qK, double rho,
                     double2* B64, float2* B32, long long* status, hipStream_t s) {
    const int64_t blocks = (g.N + TPB - 1) / TPB;
    hipLaunchKernelGGL((k_a1_solve<NT, TPB, REG>), dim3((unsigned)blocks), dim3(TPB), 0, s, g, nd, S, Ktab, qK, rho,
                       B64, B32, status);
}

}  // namespace

void launch_a1_bands(double2* out, int M, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_a1_bands, dim3((nb * M + 255) / 256), dim3(256), 0, s, out, M, nb);
}

void launch_a1_ones(double2* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_a1_ones, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n);
}

void launch_a1_products(const double2* a, double2* prod, int Ms, int d0, int nd, int npair, double scale,
                        hipStream_t s) {
    const int64_t total = (int64_t)npair * nd * Ms;
    hipLaunchKernelGGL(k_a1_products, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, prod, Ms, d0, nd,
                       npair, scale);
}

void launch_a1_fold(const double2* R, const double2* h, double2* V, int M, int Ms, int nd, int npair, hipStream_t s) {
    const int64_t total = (int64_t)nd * Ms;
    hipLaunchKernelGGL(k_a1_fold, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, R, h, V, M, Ms, nd, npair);
}

void launch_a1_solve(const Geo& g, const NodesDev& nd, const double2* S, const double2* Ktab, int qK, double rho,
                     double2* B64, float2* B32, long long* status, hipStream_t s) {
    const int n = 2 * g.m + 1;
    if (n <= 5) a1_solve_launch<5, 256, true>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
    else if (n <= 9) a1_solve_launch<9, 256, true>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
    else if (n <= 13) a1_solve_launch<13, 64, false>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
    else a1_solve_launch<17, 32, false>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
}

}  // namespace infft
