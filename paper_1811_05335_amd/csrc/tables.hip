// Node-independent tables of a plan, computed once on the device in float64:
//   * deconvolution factors D_k = 1/(M_sigma w_hat(k)) = 1/I_0(m sqrt(b^2 - (2 pi k/M_sigma)^2))
//     of (2.4) for the Kaiser-Bessel window (I_0 from its power series);
//   * FFT twiddles e^{-2 pi i e/n};
//   * Taylor tables of the kernels used by the local least-squares problems of Algorithm 3.17:
//       K(z) = sum_k D_k   e^{2 pi i k z / M_sigma}   ((3.15) in grid units z = M_sigma y)
//       Q(z) = sum_k D_k^2 e^{2 pi i k z / M_sigma}   (normal-equation kernel, G_l = M_sigma^d Q)
//     tabulated at z0 = q / TAY_S with the coefficients a_p(q) = (1/p!) sum_k c_k
//     (2 pi i k / M_sigma)^p e^{2 pi i k z0 / M_sigma}, so that F(z0 + e) = sum_p a_p(q) e^p.
//     With |e| <= 1/(2 TAY_S) each term shrinks by at least pi/(2 sigma TAY_S) <= 0.1, and ten
//     terms leave a truncation below 1e-16 of sum_k |c_k|.
#include "internal.hpp"

namespace infft {

__device__ double i0_series(double z) {
    const double q = 0.25 * z * z;
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 1000; ++n) {
        term *= q / ((double)n * (double)n);
        sum += term;
        if (term <= 1e-18 * sum) break;
    }
    return sum;
}

__global__ void k_deconv(int M, int Ms, int m, double b, double* D64, float* D32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double k = (double)(i - M / 2);
    const double w = 2.0 * M_PI * k / (double)Ms;
    const double arg = b * b - w * w;
    const double D = 1.0 / i0_series((double)m * sqrt(arg > 0.0 ? arg : 0.0));
    D64[i] = D;
    if (D32) D32[i] = (float)D;
}

void launch_deconv_table(int M, int Ms, int m, double b, double* D64, float* D32, hipStream_t s) {
    hipLaunchKernelGGL(k_deconv, dim3((M + 255) / 256), dim3(256), 0, s, M, Ms, m, b, D64, D32);
}

// t[i] = e^{-2 pi i ((i * step) mod N) / N}, the exponent reduced exactly in integers.
__global__ void k_twiddles(int64_t N, int64_t count, int64_t step, double2* t64, float2* t32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t e = (int64_t)(((__int128)i * step) % N);
    double sn, cs;
    sincospi(2.0 * (double)e / (double)N, &sn, &cs);
    t64[i] = make_double2(cs, -sn);
    if (t32) t32[i] = make_float2((float)cs, (float)-sn);
}

void launch_twiddles(int64_t n, double2* t64, float2* t32, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, n, (int64_t)1,
                       t64, t32);
}

void launch_twiddles_strided(int64_t N, int64_t count, int64_t step, double2* t64, float2* t32,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, N, count, step,
                       t64, t32);
}

// One workgroup per table row q; threads split the frequency sum, then a tree reduction.
// sym = 1 leaves out the unpaired frequency k = -M/2: the remaining sum pairs k with -k, is real
// and even in z, and only the real parts are stored (table of doubles).
__global__ void __launch_bounds__(256) k_taylor(int M, int Ms, const double* __restrict__ D, int power,
                                                double2* __restrict__ tab, int sym) {
    __shared__ double red[256];
    const int q = blockIdx.x;
    const int64_t L = (int64_t)TAY_S * Ms;   // period of the phase index
    double ax[TAY_NC], ay[TAY_NC];
#pragma unroll
    for (int p = 0; p < TAY_NC; ++p) ax[p] = ay[p] = 0.0;
    for (int i = threadIdx.x + (sym ? 1 : 0); i < M; i += blockDim.x) {
        const int64_t k = (int64_t)(i - M / 2);
        double c = D[i];
        if (power == 2) c = c * c;
        const int64_t e = (((k % L) + L) % L) * (int64_t)q % L;
        double sn, cs;
        sincospi(2.0 * (double)e / (double)L, &sn, &cs);
        const double om = 2.0 * M_PI * (double)k / (double)Ms;
        double tx = c * cs, ty = c * sn;
#pragma unroll
        for (int p = 0; p < TAY_NC; ++p) {
            ax[p] += tx;
            ay[p] += ty;
            // multiply by (i om) / (p+1)
            const double f = om / (double)(p + 1);
            const double nx = -ty * f, ny = tx * f;
            tx = nx;
            ty = ny;
        }
    }
#pragma unroll
    for (int p = 0; p < 2 * TAY_NC; ++p) {
        if (sym && (p & 1)) continue;
        red[threadIdx.x] = (p & 1) ? ay[p >> 1] : ax[p >> 1];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (sym) {
                ((double*)tab)[(int64_t)q * TAY_NC + (p >> 1)] = red[0];
            } else {
                double2* dst = &tab[(int64_t)q * TAY_NC + (p >> 1)];
                if (p & 1) dst->y = red[0];
                else dst->x = red[0];
            }
        }
        __syncthreads();
    }
}

void launch_taylor_table(int M, int Ms, const double* D, int power, int qmax, double2* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_taylor, dim3(qmax + 1), dim3(256), 0, s, M, Ms, D, power, tab, 0);
}

void launch_taylor_table_sym(int M, int Ms, const double* D, int power, int qmax, double* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_taylor, dim3(qmax + 1), dim3(256), 0, s, M, Ms, D, power, (double2*)tab, 1);
}

}  // namespace infft
