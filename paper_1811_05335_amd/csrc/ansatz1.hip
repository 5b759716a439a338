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
// R_d comes from grid samples: with a^lo, a^hi the two half-band parts of K on the grid
// (a^b[s] = sum_{k in b} D_k e^{2 pi i k s / M_sigma}), conj(a^b[s]) a^c[s - d] holds the
// frequencies q = k' - k of R_d restricted to k in b, k' in c, a range of width < M <= M_sigma,
// so its length-M_sigma DFT gives them without aliasing for every sigma >= 1.  This replaces the
// paper's N NFFTs of length N(2m+1) (O(N^2)) by O(m M_sigma log M_sigma) FFT work and one
// adjoint NFFT of bandwidth 2M for P.
//
// All arithmetic here is FP64.  The host side (abi.cpp) runs the FFTs and the adjoint NFFT.

#include "internal.hpp"

namespace infft {
namespace {

// The two half bands of the coefficient range as FFT inputs: [2][M], band 0 is k < 0, band 1 k >= 0.
__global__ void k_a1_bands(double2* __restrict__ out, int M) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * M) return;
    const int band = i / M, k = i - band * M;     // k is the centred index + M/2
    const bool on = (band == 0) ? (k < M / 2) : (k >= M / 2);
    out[i] = make_double2(on ? 1.0 : 0.0, 0.0);
}

__global__ void k_a1_ones(double2* __restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_double2(1.0, 0.0);
}

// prod[c][dd][s] = conj(a^b[s]) a^b'[(s - d) mod M_sigma] * scale for the pairs
// c = (lo,lo), (hi,hi), (lo,hi), (hi,lo) and d = d0 + dd.
__global__ void k_a1_products(const double2* __restrict__ a, double2* __restrict__ prod, int Ms, int d0, int nd,
                              double scale) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)4 * nd * Ms;
    if (i >= total) return;
    const int s = (int)(i % Ms);
    const int64_t r = i / Ms;
    const int dd = (int)(r % nd);
    const int c = (int)(r / nd);
    const int bl = (c == 1 || c == 3) ? 1 : 0;   // band of k
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
                          int M, int Ms, int nd) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nd * Ms) return;
    const int r = (int)(i % Ms);
    const int dd = (int)(i / Ms);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int lo = c < 2 ? -(M / 2 - 1) : (c == 2 ? 1 : -(M - 1));
        const int hi = c < 2 ? (M / 2 - 1) : (c == 2 ? (M - 1) : -1);
        const int q = r <= hi ? r : r - Ms;
        if (q < lo || q > hi) continue;
        const double2 p = h[M - q];
        const double2 v = R[((int64_t)c * nd + dd) * Ms + r];
        acc.x += p.x * v.x - p.y * v.y;
        acc.y += p.x * v.y + p.y * v.x;
    }
    V[i] = acc;
}

inline __device__ int tri(int a, int b) { return a * (a + 1) / 2 + b; }

// One thread per node (sorted order).  The Hermitian system over the 2m+1 taps keeps identity
// rows for taps outside I(x_j), so their entries come out zero; packed lower triangle in LDS,
// one column per thread.  B_opt^* column j is stored as rows[tau][p] = conj(y_tau), which makes
// the modified adjoint D^* F^* B^* f equal (1/M) D^* F^* B_opt^* f of the paper.
template <int NT, int TPB, typename R2>
__global__ __launch_bounds__(TPB) void k_a1_solve(Geo g, NodesDev nd, const double2* __restrict__ S,
                                                  const double2* __restrict__ Ktab, int qK, double rho,
                                                  double2* __restrict__ B64, R2* __restrict__ Blo,
                                                  long long* __restrict__ status) {
    constexpr int NE = NT * (NT + 1) / 2;
    __shared__ double2 s_A[NE][TPB];
    __shared__ unsigned long long s_mn, s_mx, s_fail;
    const int t = threadIdx.x;
    if (t == 0) {
        s_mn = ~0ull;
        s_mx = 0ull;
        s_fail = 0ull;
    }
    __syncthreads();
    const int64_t p = blockIdx.x * (int64_t)TPB + t;
    const int Ms = g.Ms[0], m = g.m;
    const int n = 2 * m + 1;
    if (p < g.N) {
        const int l0 = nd.l0s[p];
        const double u = nd.us[p];
        bool mem[NT];
        int cnt = 0;
        double tr = 0.0;
        double2 y[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            mem[a] = a < n && isfinite(u) && (a < 2 * m || edge_tap_member(u, m));
            y[a] = make_double2(0.0, 0.0);
            if (mem[a]) {
                ++cnt;
                int la = l0 + a;
                if (la >= Ms) la -= Ms;
                tr += S[la].x;
                // K_j^* e_j entry: conj K((u - tau)/M_sigma) = K((tau - u)/M_sigma)
                y[a] = tay_eval(Ktab, qK, (double)a - u);
            }
        }
        const double lam = cnt > 0 ? rho * tr / (double)cnt : 0.0;
        // Gram: entry (a, b), a >= b, is (K^* K)[l_a, l_b] = conj S(l_b, a - b)
#pragma unroll
        for (int a = 0; a < NT; ++a) {
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                double2 v = make_double2(0.0, 0.0);
                if (mem[a] && mem[b]) {
                    int lb = l0 + b;
                    if (lb >= Ms) lb -= Ms;
                    const double2 sv = S[(int64_t)(a - b) * Ms + lb];
                    v = make_double2(sv.x, a == b ? 0.0 : -sv.y);
                    if (a == b) v.x += lam;
                } else if (a == b) {
                    v.x = 1.0;
                }
                s_A[tri(a, b)][t] = v;
            }
        }
        // Cholesky A = L L^*; the reciprocal of each pivot replaces it on the diagonal
        bool ok = cnt > 0;
        for (int j = 0; j < NT && ok; ++j) {
            double sd = s_A[tri(j, j)][t].x;
            for (int k = 0; k < j; ++k) {
                const double2 l = s_A[tri(j, k)][t];
                sd -= l.x * l.x + l.y * l.y;
            }
            if (!(sd > 0.0)) {
                ok = false;
                break;
            }
            const double inv = 1.0 / sqrt(sd);
            s_A[tri(j, j)][t] = make_double2(inv, 0.0);
            for (int i = j + 1; i < NT; ++i) {
                double2 v = s_A[tri(i, j)][t];
                for (int k = 0; k < j; ++k) {
                    const double2 li = s_A[tri(i, k)][t], lj = s_A[tri(j, k)][t];
                    // v -= L[i][k] conj(L[j][k])
                    v.x -= li.x * lj.x + li.y * lj.y;
                    v.y -= li.y * lj.x - li.x * lj.y;
                }
                s_A[tri(i, j)][t] = make_double2(v.x * inv, v.y * inv);
            }
        }
        if (ok) {
            // L z = r, then L^* y = z
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                double2 v = y[i];
#pragma unroll
                for (int k = 0; k < i; ++k) {
                    const double2 l = s_A[tri(i, k)][t];
                    v.x -= l.x * y[k].x - l.y * y[k].y;
                    v.y -= l.x * y[k].y + l.y * y[k].x;
                }
                const double inv = s_A[tri(i, i)][t].x;
                y[i] = make_double2(v.x * inv, v.y * inv);
            }
#pragma unroll
            for (int i = NT - 1; i >= 0; --i) {
                double2 v = y[i];
#pragma unroll
                for (int k = i + 1; k < NT; ++k) {
                    const double2 l = s_A[tri(k, i)][t];   // conj(L[k][i]) y_k
                    v.x -= l.x * y[k].x + l.y * y[k].y;
                    v.y -= l.x * y[k].y - l.y * y[k].x;
                }
                const double inv = s_A[tri(i, i)][t].x;
                y[i] = make_double2(v.x * inv, v.y * inv);
            }
        } else {
#pragma unroll
            for (int a = 0; a < NT; ++a) y[a] = make_double2(0.0, 0.0);
            if (cnt > 0) atomicAdd(&s_fail, 1ull);
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            if (a >= n) continue;
            const double2 v = mem[a] ? make_double2(y[a].x, -y[a].y) : make_double2(0.0, 0.0);
            B64[(int64_t)a * g.N + p] = v;
            if (Blo) Blo[(int64_t)a * g.N + p] = R2{(float)v.x, (float)v.y};
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

template <int NT, int TPB>
void a1_solve_launch(const Geo& g, const NodesDev& nd, const double2* S, const double2* Ktab, int qK, double rho,
                     double2* B64, float2* B32, long long* status, hipStream_t s) {
    const int64_t blocks = (g.N + TPB - 1) / TPB;
    hipLaunchKernelGGL((k_a1_solve<NT, TPB, float2>), dim3((unsigned)blocks), dim3(TPB), 0, s, g, nd, S, Ktab, qK,
                       rho, B64, B32, status);
}

}  // namespace

void launch_a1_bands(double2* out, int M, hipStream_t s) {
    hipLaunchKernelGGL(k_a1_bands, dim3((2 * M + 255) / 256), dim3(256), 0, s, out, M);
}

void launch_a1_ones(double2* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_a1_ones, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n);
}

void launch_a1_products(const double2* a, double2* prod, int Ms, int d0, int nd, double scale, hipStream_t s) {
    const int64_t total = (int64_t)4 * nd * Ms;
    hipLaunchKernelGGL(k_a1_products, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, prod, Ms, d0, nd,
                       scale);
}

void launch_a1_fold(const double2* R, const double2* h, double2* V, int M, int Ms, int nd, hipStream_t s) {
    const int64_t total = (int64_t)nd * Ms;
    hipLaunchKernelGGL(k_a1_fold, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, R, h, V, M, Ms, nd);
}

void launch_a1_solve(const Geo& g, const NodesDev& nd, const double2* S, const double2* Ktab, int qK, double rho,
                     double2* B64, float2* B32, long long* status, hipStream_t s) {
    const int n = 2 * g.m + 1;
    if (n <= 5) a1_solve_launch<5, 64>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
    else if (n <= 9) a1_solve_launch<9, 64>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
    else if (n <= 13) a1_solve_launch<13, 64>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
    else a1_solve_launch<17, 32>(g, nd, S, Ktab, qK, rho, B64, B32, status, s);
}

}  // namespace infft
