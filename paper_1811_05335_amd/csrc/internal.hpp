// Internal declarations shared by the HIP translation units of libinfft.
//
// Grid conventions (Section 2.1 of the paper, tensor product for d = 2):
//   grid index l_t in 0..M_sigma_t-1 (l mod M_sigma, FFT storage order), row-major over
//   dimensions (dimension 0 slowest).  Coefficients are centred: index k_t + M_t/2.
//   Node stencil per dimension: t = x M_sigma, l0 = ceil(t - m), u = t - l0 in (m-1, m];
//   taps tau = 0..2m reach grid index (l0 + tau) mod M_sigma with window argument u - tau;
//   a tap is inside the truncated window when |u - tau| <= m.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace infft {

// Pointers read from device memory (the job tables of the batch kernels) are generic to the
// compiler, which then emits flat instructions, whose completion is counted with the LDS operations
// (an LDS wait also waits for them).  Accesses to arrays that always lie in global memory go
// through this cast and become global instructions.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> glb(T* p) { return (gptr<T>)p; }

// ------------------------------------------------------------------ complex helpers

template <typename R> struct CxT;
template <> struct CxT<float> { using T = float2; };
template <> struct CxT<double> { using T = double2; };
template <typename R> using cx = typename CxT<R>::T;

__host__ __device__ inline float2 cmake(float a, float b) { return make_float2(a, b); }
__host__ __device__ inline double2 cmake(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ------------------------------------------------------------------ plan geometry

constexpr int MAX_D = 2;
constexpr int MIN_M_CUT = 2;
constexpr int MAX_M_CUT = 8;   // window cut-off m supported by the compiled kernels
constexpr int STATUS_WORDS = 8;
enum StatusWord {
    ST_NONFINITE = 0,
    ST_FAILED = 1,
    ST_EMPTY = 2,
    ST_OVERSIZED = 3,
    ST_MIN_N = 4,
    ST_MAX_N = 5,
};

struct Geo {
    int d;
    int m;
    int M[MAX_D];      // coefficients per dimension (1 for unused dimensions)
    int Ms[MAX_D];     // oversampled grid per dimension (1 for unused dimensions)
    int TS[MAX_D];     // spreading tile, cells per dimension (1 for unused dimensions)
    int ntile[MAX_D];  // Ms / TS
    int64_t N;
    int64_t G;         // prod Ms
    int64_t P;         // prod M
    double b;          // Kaiser-Bessel shape pi (2 - 1/sigma)
    // Window polynomials: for a node with offset u in (m-1, m], tap tau < 2m lies in one unit
    // interval of the window, w(u - tau) = P_tau(y) with y = 2 (u - (m-1)) - 1 in [-1, 1];
    // coefficients (plan precision) [tau][WPOLY_NC], ascending powers of y.
    const void* wpoly;
};
template <typename R> struct WPoly;
template <> struct WPoly<float> { static constexpr int NC = 11; };   // degree 10: ~2e-7 relative
template <> struct WPoly<double> { static constexpr int NC = 17; };  // degree 16: ~2e-14 relative

// Sort key of grid cell (c0, c1): tile-major, row-major inside a tile, so that the nodes of one
// spreading tile form a contiguous range in sorted order.
__host__ __device__ inline int64_t cell_key(const Geo& g, int c0, int c1) {
    if (g.d == 1) return c0;
    const int t0 = c0 / g.TS[0], t1 = c1 / g.TS[1];
    const int o0 = c0 - t0 * g.TS[0], o1 = c1 - t1 * g.TS[1];
    return ((int64_t)t0 * g.ntile[1] + t1) * ((int64_t)g.TS[0] * g.TS[1]) + (int64_t)o0 * g.TS[1] + o1;
}

// Tap 2m of a node with offset u in (m-1, m] is inside the closed window support when
// |u - 2m| <= m in FP64: at u = m exactly, and also when u lies within rounding of m (the
// difference then rounds to -m).  Every kernel takes this decision in this one way.
__host__ __device__ inline bool edge_tap_member(double u, int m) {
    return fabs(u - 2.0 * (double)m) <= (double)m;
}

// One entry of B_opt: the FP64 copy and the FP32 copy, each where the launch writes it (an FP32
// plan's B optimisation writes only the FP32 copy; its FP64 values are recomputed on demand).
__device__ inline void put_bopt(double2* B64, float2* B32, int64_t idx, double2 v) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    typedef float f2v __attribute__((ext_vector_type(2)));
    if (B64) *(gptr<d2v>)(B64 + idx) = d2v{v.x, v.y};
    if (B32) *(gptr<f2v>)(B32 + idx) = f2v{(float)v.x, (float)v.y};
}

struct NodesDev {
    const double* xw;  // [N][d] wrapped nodes, caller order
    int* l0c;          // [N][d] stencil base mod M_sigma, caller order
    double* uc;        // [N][d] offsets u = x M_sigma - l0, caller order
    int* key;          // [N]    cell key per node, caller order
    int* perm;         // [N]    sorted position -> caller index
    int* l0s;          // [N][d] stencil base, sorted order
    double* us;        // [N][d] offsets, sorted order
    int* start;        // [G+1]  CSR over cell keys: nodes of key c are start[c]..start[c+1)-1
};

// Taylor tables of the kernels K (coefficients D_k) and Q (coefficients D_k^2), per dimension,
// on the grid z = q / TAY_S (grid units), q = 0..qmax; negative arguments use conjugate symmetry.
constexpr int TAY_S = 16;
constexpr int TAY_NC = 10;
struct KTabDev {
    const double2* K[MAX_D];
    const double2* Q[MAX_D];
    // 1-D split K = Ks + d e^{-i pi z / sigma}, Q = Qs + d^2 e^{-i pi z / sigma}: Ks, Qs are the
    // real, even sums over the frequency pairs +-k; d = D_{-M/2} is the unpaired frequency
    const double* Ks;
    const double* Qs;
    double dM;         // D_{-M/2}
    double inv_sigma;  // M / M_sigma
    int qK, qQ;        // largest table index for K and Q
    double lam;        // ridge lambda (the same for every l: all diagonal entries of G_l agree)
    double scaleG;     // prod M_sigma
};

// Taylor evaluation of a complex kernel table at z (grid units); the tables hold z >= 0 and
// F(-z) = conj F(z) because the coefficients D_k are real.
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

// ------------------------------------------------------------------ members of I(l) for lane groups

// Ordering point for the LDS exchange inside one wavefront: LDS operations of a wave execute
// in program order, so only the compiler has to be kept from moving accesses across it.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Members of I(l) for d = 1.  Nodes are sorted by stencil base l0, so the cells l-2m+1 .. l
// (every node of them reaches l) form at most two contiguous ranges of the sorted order (two when
// the window wraps around the torus); the cell l-2m contributes only nodes whose tap 2m is a member.
__device__ inline void gather_1d(const Geo& g, const NodesDev& nd, int l, int lane, int NL, int gbase,
                                 uint64_t gmask, int& n, int& my_p) {
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
    if (lane < n0) my_p = s0 + lane;
    else if (lane - n0 < n1) my_p = s1 + (lane - n0);
    n = n0 + n1;
    int ce = l - w2;
    if (ce < 0) ce += Ms;
    const int s = glb(nd.start)[ce], e = glb(nd.start)[ce + 1];
    for (int base = s; base < e; base += NL) {
        const int p = base + lane;
        const bool mem = p < e && edge_tap_member(glb(nd.us)[p], g.m);
        const uint64_t gm = (__ballot(mem) >> gbase) & gmask;
        const int cnt = __popcll(gm);
        const int k = lane - n;
        if (k >= 0 && k < cnt) {
            uint64_t mm = gm;
            for (int i = 0; i < k; ++i) mm &= mm - 1ull;
            my_p = base + (__ffsll((unsigned long long)mm) - 1);
        }
        n += cnt;
    }
}

// Members of I(l) for d = 2: the (2m+1)^2 cells (l0 - tau0, l1 - tau1), cell by cell.
__device__ inline void gather_2d(const Geo& g, const NodesDev& nd, int l, int lane, int NL, int gbase,
                                 uint64_t gmask, int& n, int& my_p) {
    const int W = 2 * g.m + 1, w2 = 2 * g.m;
    const int lc0 = l / g.Ms[1], lc1 = l - lc0 * g.Ms[1];
    n = 0;
    for (int c = 0; c < W * W; ++c) {
        const int tau0 = c / W, tau1 = c - tau0 * W;
        int c0 = lc0 - tau0;
        if (c0 < 0) c0 += g.Ms[0];
        int c1 = lc1 - tau1;
        if (c1 < 0) c1 += g.Ms[1];
        const int64_t key = cell_key(g, c0, c1);
        const int s = nd.start[key], e = nd.start[key + 1];
        if (s == e) continue;
        if (tau0 < w2 && tau1 < w2) {
            const int k = lane - n;
            if (k >= 0 && k < e - s) my_p = s + k;
            n += e - s;
        } else {
            for (int base = s; base < e; base += NL) {
                const int p = base + lane;
                bool mem = p < e;
                if (mem && tau0 == w2) mem = edge_tap_member(nd.us[(int64_t)p * 2], g.m);
                if (mem && tau1 == w2) mem = edge_tap_member(nd.us[(int64_t)p * 2 + 1], g.m);
                const uint64_t gm = (__ballot(mem) >> gbase) & gmask;
                const int cnt = __popcll(gm);
                const int k = lane - n;
                if (k >= 0 && k < cnt) {
                    uint64_t mm = gm;
                    for (int i = 0; i < k; ++i) mm &= mm - 1ull;
                    my_p = base + (__ffsll((unsigned long long)mm) - 1);
                }
                n += cnt;
            }
        }
    }
}


// ------------------------------------------------------------------ large local problems

constexpr int BIG_NB = 64;   // block size of the blocked Cholesky

struct BigProb {
    int l;         // grid index
    int n;         // members |I(l)|
    int nblk;      // ceil(n / BIG_NB)
    int id;        // index of the problem's failure flag
    int64_t off;   // first entry of its n x n matrix (row-major) in the workspace
    int64_t moff;  // first member slot
};

struct BigArgs {
    const BigProb* probs;
    double2* A;    // Gram matrices, then their Cholesky factors (lower triangle; the strictly
                   // upper part of each diagonal block holds its inverse, conjugate-transposed)
    int* midx;     // member -> sorted node position
    int* mtap;     // member -> tap index (row of B_opt)
    double2* mz;   // member -> z = tau - u per dimension
    double2* mr;   // member -> right-hand side, then solution
    double2* mb;   // member -> its B_opt entry (node gradient pass)
    int* fail;     // per problem id: non-positive pivot
    const int* stale;   // device flag: the recorded problems do not match the current lists, so
                        // every large-problem kernel returns at once (nullptr: never)
};

constexpr int BIG_TPB = 256;   // threads of the large-problem kernels

// X[c][q] = (L_kk^{-1})[c][q] from the diagonal block D of the factor.
__device__ inline double2 inv_entry(const double2* D, int64_t ld, int c, int q) {
    if (q < c) return cconj(D[(int64_t)q * ld + c]);
    if (q == c) return make_double2(1.0 / D[(int64_t)c * ld + c].x, 0.0);
    return make_double2(0.0, 0.0);
}

// Solves (L L^*) x = y in place for one large problem (the whole workgroup; y in device memory,
// read and written between barriers by this workgroup only), with the factor of k_big_potrf..herk.
__device__ inline void big_substitute(const BigProb& P, const double2* A, double2* y, int nblk) {
    constexpr int NP = BIG_TPB / BIG_NB;
    __shared__ double2 s_t[BIG_NB];
    __shared__ double2 red[NP][BIG_NB];
    const int64_t ld = P.n;
    const int col = threadIdx.x % BIG_NB, part = threadIdx.x / BIG_NB;
    // ---- L y = r: y_k = X_k (r_k - sum_{c < r0} L[r0 + i][c] y_c)
    for (int k = 0; k < nblk; ++k) {
        const int r0 = k * BIG_NB, nk = min(BIG_NB, P.n - r0);
        const int i = threadIdx.x / NP, p4 = threadIdx.x % NP;   // NP threads per row
        double2 acc = make_double2(0.0, 0.0);
        if (i < nk) {
            const double2* row = A + (int64_t)(r0 + i) * ld;
            for (int c = p4; c < r0; c += NP) acc = cadd(acc, cmul(row[c], y[c]));
        }
#pragma unroll
        for (int o = 1; o < NP; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (p4 == 0 && i < nk) s_t[i] = csub(y[r0 + i], acc);
        __syncthreads();
        const double2* D = A + (int64_t)r0 * ld + r0;
        double2 v = make_double2(0.0, 0.0);
        if (i < nk)
            for (int c = p4; c <= i; c += NP) v = cadd(v, cmul(inv_entry(D, ld, i, c), s_t[c]));
#pragma unroll
        for (int o = 1; o < NP; o <<= 1) {
            v.x += __shfl_xor(v.x, o, 64);
            v.y += __shfl_xor(v.y, o, 64);
        }
        if (p4 == 0 && i < nk) y[r0 + i] = v;
        __syncthreads();
    }
    // ---- L^* b = y: b_k = X_k^* (y_k - sum_{i >= r0 + nk} conj(L[i][r0 + c]) b_i)
    for (int k = nblk - 1; k >= 0; --k) {
        const int r0 = k * BIG_NB, nk = min(BIG_NB, P.n - r0);
        double2 acc = make_double2(0.0, 0.0);
        if (col < nk)
            for (int i = r0 + nk + part; i < P.n; i += NP) acc = cadd(acc, cmul(cconj(A[(int64_t)i * ld + r0 + col]), y[i]));
        red[part][col] = acc;
        __syncthreads();
        if (part == 0 && col < nk) {
            double2 s = red[0][col];
            for (int pp = 1; pp < NP; ++pp) s = cadd(s, red[pp][col]);
            s_t[col] = csub(y[r0 + col], s);
        }
        __syncthreads();
        const double2* D = A + (int64_t)r0 * ld + r0;
        double2 v = make_double2(0.0, 0.0);
        if (col < nk)
            for (int r = col + part; r < nk; r += NP) v = cadd(v, cmul(cconj(inv_entry(D, ld, r, col)), s_t[r]));
        red[part][col] = v;
        __syncthreads();
        if (part == 0 && col < nk) {
            double2 s = red[0][col];
            for (int pp = 1; pp < NP; ++pp) s = cadd(s, red[pp][col]);
            y[r0 + col] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ FFT pass description

constexpr int FFT_THREADS = 512;

// Workgroups of a launch go to the eight XCDs (each with its own L2) in turn: workgroup b runs on
// XCD b mod 8.  This maps the launch index to a logical block so that each XCD takes one
// contiguous range of logical blocks (a bijection on [0, n)): neighbouring blocks, which read the
// same cache lines of a strided pass, then share one L2 instead of fetching the lines eight times.
constexpr int NUM_XCD = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t n) {
    const int64_t per = n / NUM_XCD, rem = n % NUM_XCD;
    const int64_t x = b % NUM_XCD, k = b / NUM_XCD;
    return x * per + (x < rem ? x : rem) + k;
}
constexpr int FFT_MAX_STAGES = 16;
enum LoadMode { LD_GRID = 0, LD_DECONV = 1, LD_HALO = 2 };
enum StoreMode { ST_GRID = 0, ST_TWIDDLE = 1, ST_DECONV = 2 };

struct FftPass {
    int n;             // sub-transform length
    int rows;          // sub-transforms per workgroup
    int nst;           // number of Stockham stages
    int rad[FFT_MAX_STAGES];
    int sign;          // exponent sign: +1 (F) or -1 (F^*)
    int64_t nq;        // sub-transforms per right-hand side
    int64_t nseq;      // total sub-transforms (nq * nrhs)
    int64_t in_rs, in_qs, in_is;    // input offset  = r*in_rs + q*in_qs + i*in_is
    int64_t out_rs, out_qs, out_ks; // output offset = r*out_rs + q*out_qs + k*out_ks
    int in_rowfast, out_rowfast;    // thread mapping for coalescing
    const void* tw;    // e^{-2 pi i e / n}, e = 0..n-1
    // inter-pass twiddle omega_N^{sign * q * k}, from two tables: e = hi * twB + lo
    int64_t twN;
    int twB;           // a power of two, 1 << twShift
    int twShift;
    const void* twLo;  // e^{-2 pi i lo / N}, lo < twB
    const void* twHi;  // e^{-2 pi i hi twB / N}
};

struct FftIO {
    const void* in;
    void* out;
    const void* D0;    // deconvolution factors (plan precision), length M0
    const void* D1;    // length M1 (d = 2)
    const void* h0;    // halo overflowing dimension 0: [r][tile][2m][TS1]
    const void* h1;    // halo overflowing dimension 1: [r][tile][TS0][2m]
    const void* h01;   // corner: [r][tile][2m][2m]
    int64_t halo_rs0, halo_rs1, halo_rs01;  // per right-hand side strides of the halos
};

// One problem's share of a batched launch: the pass (or kernel arguments) of that problem, and
// where its caller-side array starts inside the batch array (problem-major: nrhs * user_off).
struct FftJob {
    FftPass pass;
    FftIO io;
    Geo g;
    int user_in, user_out;   // the pass reads / writes the caller's array
    int64_t user_off;        // the problem's first element (per right-hand side) in the batch
};

// Per-node and per-cell kernels of one 1-D problem inside a batch.
struct NodeJob {
    Geo g;
    NodesDev nd;
    const void* B;      // B_opt of the problem ([tap][N_i], sorted order, plan precision)
    void* grid;         // the problem's oversampled grid, [rhs][M_sigma_i]
    int64_t grs;        // grid stride per right-hand side
    int64_t noff;       // first node of the problem in the batch
};
enum NodeBatchKind { NB_INTERP = 0, NB_INTERP_B = 1, NB_GATHER = 2, NB_GATHER_B = 3, NB_GRAD = 4 };

// ------------------------------------------------------------------ launchers (per .hip file)

// nodes.hip
void launch_fill_i32(int* p, int64_t n, int v, hipStream_t s);
void launch_fill_bytes0(void* p, int64_t nbytes, hipStream_t s);
void launch_prep_nodes(const Geo& g, const double* x, NodesDev nd, int* counts, int* nonfinite, hipStream_t s);
int prep_blocks(const Geo& g);
void launch_exclusive_scan(const int* in, int* out, int64_t n, int* blocksums, hipStream_t s);
int64_t scan_blocksum_len(int64_t n);
// counting sort by cell after launch_prep_nodes (scan, scatter, in-cell sort; writes nd.start)
void launch_sort_nodes(const Geo& g, NodesDev nd, int* counts, int* fill, int* bsum, const int* nonfinite,
                       long long* status, hipStream_t s);
void launch_export_B(const Geo& g, const int* perm, const double2* B, double2* rows, hipStream_t s);
void launch_status_init(long long* status, int keep_node_words, hipStream_t s);
void launch_nodes_reset(long long* status, int* counts, int64_t ncounts, int* fill, int64_t nfill, int* lcount,
                        hipStream_t s);

// tables.hip
void launch_deconv_table(int M, int Ms, int m, double b, double* D64, float* D32, hipStream_t s);
void launch_twiddles(int64_t n, double2* t64, float2* t32, hipStream_t s);
void launch_twiddles_strided(int64_t N, int64_t count, int64_t step, double2* t64, float2* t32,
                             hipStream_t s);
void launch_taylor_table(int M, int Ms, const double* D, int power, int qmax, double2* tab,
                         hipStream_t s);
void launch_taylor_table_sym(int M, int Ms, const double* D, int power, int qmax, double* tab,
                             hipStream_t s);

// fft.hip
template <typename R>
void launch_fft_pass(const FftPass& p, const FftIO& io, const Geo& g, int ld, int st, hipStream_t s);
int fft_capacity(bool fp64);   // elements of one workgroup's LDS transform buffer
int fft_batched_small_capacity();   // elements per workgroup of the small batched FP32 pass kernel
size_t fft_lds_bytes(const FftPass& p, size_t csize);   // LDS of one pass's workgroup (data + twiddles)
template <typename R>
void launch_fft_batched(const FftJob* jobs, const int2* bmap, int nblocks, size_t shm, int ld, int st,
                        const void* user_in, void* user_out, int nrhs, bool small, hipStream_t s);

// spread.hip
template <typename R>
void launch_interp(const Geo& g, NodesDev nd, const cx<R>* grid, int64_t grid_rs, cx<R>* f,
                   int nrhs, hipStream_t s);
// Work list of the 2-D tiled spreading (built at node preprocessing): items (tile, chunk) with at
// most `chunk` nodes each; tiles split into several chunks flush with atomics.
struct SpreadWork {
    int chunk;       // nodes per work item
    int cap;         // capacity of items (launch size; items beyond *total exit)
    int* nchunk;     // [ntiles]
    int2* items;     // [cap]
    int* total;      // number of items
};
void launch_spread_worklist(const Geo& g, NodesDev nd, SpreadWork wk, int* offs, int* bsum, hipStream_t s);
template <typename R>
void launch_spread(const Geo& g, NodesDev nd, const cx<R>* f, const cx<R>* B, cx<R>* grid,
                   int64_t grid_rs, cx<R>* h0, cx<R>* h1, cx<R>* h01, int64_t hrs0, int64_t hrs1,
                   int64_t hrs01, int nrhs, int rchunk, SpreadWork wk, hipStream_t s);
template <typename R>
void launch_interp_B(const Geo& g, NodesDev nd, const cx<R>* grid, int64_t grid_rs, const cx<R>* B,
                     cx<R>* f, int nrhs, hipStream_t s);
template <typename R>
void launch_grad_x(const Geo& g, NodesDev nd, const cx<R>* grid, int64_t grid_rs, const cx<R>* gradf,
                   double* gradx, int nrhs, int accumulate, hipStream_t s);
int spread_rhs_chunk(const Geo& g);
int spread1d_tiles(const Geo& g);   // workgroups of the tiled 1-D spreading
// kind NB_*: interpolation reads the grid and writes `out`; gathers read `in` and write the grid;
// the gradient reads `in` (gradient of f) and writes `gradx`
template <typename R>
void launch_node_batched(int kind, int m, const NodeJob* jobs, const int2* bmap, int nblocks, const cx<R>* in,
                         cx<R>* out, double* gradx, int nrhs, int accumulate, hipStream_t s);

// solve.hip
struct SolveArgs {
    const int* in_list;     // nullptr: all grid indices in order
    const int* in_count;
    int* out_list;          // problems too large for this tier
    int* out_count;
    int* out_list2;         // thread tier of a batch: problems of 17 to 32 members (count exact) go
    int* out_count2;        // here, past the 16-lane tier (nullptr: all go to out_list)
    double2* B64;           // [T][N] sorted order (nullptr: the B optimisation of an FP32 plan)
    float2* B32;            // [T][N] sorted order (nullptr: FP64 plans, and an FP32 plan's FP64 recompute)
    long long* status;
    long long* stat_rec;    // per-block statistics records [block][5]
    int stat_off;           // first record of this launch
    int tables_in_lds;      // set by the launcher (1-D plans whose kernel tables fit in LDS)
    long long* rec0;        // first tier of a B optimisation: statistics record 0 to reset (else nullptr)
    int* zero0;             // list counters this launch clears (workgroup 0) for a later launch: ones
    int* zero1;             // no kernel reads any more, in place of a reset launch (nullptr: none)
};
int launch_solve_tier(const Geo& g, NodesDev nd, KTabDev kt, SolveArgs a, int nl, hipStream_t s);
// One 1-D problem of a batch for the solve kernels (its own tables, lists and statistics slots).
struct SolveJob {
    Geo g;
    NodesDev nd;
    KTabDev kt;
    SolveArgs a;
};
// Thread-per-problem tier over all problems of a batch (workgroup -> (job, block of 128 cells)).
void launch_solve_t1_batched(const SolveJob* jobs, const int2* t1_map, int t1_blocks, int qQ, int qK,
                             hipStream_t s);
void launch_batch_solve_reset(const SolveJob* jobs, int njobs, hipStream_t s);
void launch_batch_counts(const SolveJob* jobs, int njobs, int* out, hipStream_t s);
constexpr int T1_CELLS = 256;   // cells per workgroup of the thread-per-problem tier
// Group tier (nl = 16, 32 or 64) over the lists of all problems of a batch as one flat list.
void launch_solve_tier_batched(const SolveJob* jobs, int njobs, int nl, int blocks, hipStream_t s);
int launch_solve_thread_1d(const Geo& g, NodesDev nd, KTabDev kt, SolveArgs a, hipStream_t s);
void launch_solve_stats(const long long* rec, int nrec, long long* status, hipStream_t s);

// grad_bopt.hip: node gradient through B_opt(x)
struct BoptGradArgs {
    const double2* B64;   // B_opt [tap][N] (sorted order)
    const void* grid;     // upstream grid gradient F D gfc, [R][G] (plan precision)
    const void* f;        // samples [R][N] (caller order, plan precision)
    int nrhs;
    double* gradx;        // [N][d] (caller order), accumulated with atomics
    const int* in_list;   // nullptr: all grid indices
    const int* in_count;
    int* out_list;        // problems with more members than the tier's lanes
    int* out_count;
};
template <typename R>
int launch_bopt_grad(const Geo& g, NodesDev nd, KTabDev kt, BoptGradArgs ga, int nl, hipStream_t s);
// the same for a batch of large problems, on factors from the blocked Cholesky pass
void launch_big_grad(const Geo& g, BigArgs a, KTabDev kt, BoptGradArgs ga, const int* perm, int nprob, bool f32,
                     hipStream_t s);

// solve_big.hip
void launch_big_count(const Geo& g, NodesDev nd, const int* list, int count, int* nout, hipStream_t s);
void launch_big_setup(const Geo& g, NodesDev nd, KTabDev kt, BigArgs a, int nprob, hipStream_t s);
void launch_big_gram(const Geo& g, KTabDev kt, BigArgs a, const int4* tasks, int ntask, hipStream_t s);
void launch_big_potrf(BigArgs a, int nprob, int k, hipStream_t s);
void launch_big_trsm(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s);
void launch_big_herk(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s);
void launch_big_solve(const Geo& g, BigArgs a, int nprob, double2* B64, float2* B32, hipStream_t s);
void launch_big_fwd(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s);
void launch_big_bwd(BigArgs a, const int4* tasks, int ntask, int k, hipStream_t s);
void launch_big_write(const Geo& g, BigArgs a, int nprob, double2* B64, float2* B32, hipStream_t s);
void launch_big_stats(const int* fail, int n, int nmin, int nmax, long long* rec, hipStream_t s);
// slot[probs[i].l] = i for the recorded problems (slot cleared to -1 beforehand)
void launch_big_slots(const BigProb* probs, int count, int* slot, hipStream_t s);
// Compares the device list of problems beyond the register tiers (count on the device) with the
// record of generation `gen`: stale[1] must still hold gen (no newer record), the count must match
// and every listed grid index be recorded with the same |I(l)|; any difference sets stale[0]
// (cleared by the caller beforehand).
void launch_big_check(const Geo& g, NodesDev nd, const int* list, const int* count, const int* slot,
                      const BigProb* probs, int rec_count, int gen, int* stale, hipStream_t s);
// A record without problems, replayed: if the tiers list any problem or *gen_dev is no longer
// gen, zero the listed problems' B_opt entries (1-D) and count them as oversized in statistics
// record 0, in one launch.
void launch_big_guard_empty(const Geo& g, NodesDev nd, const int* list, const int* count, const int* gen_dev, int gen,
                            double2* B64, float2* B32, long long* rec0, long long* status, hipStream_t s);
// When *stale: zero the B_opt entries of every listed problem (1-D; 2-D columns start zeroed) and
// count the listed problems as oversized in statistics record 0.
void launch_big_zero_stale(const Geo& g, NodesDev nd, const int* list, const int* count, const int* stale,
                           double2* B64, float2* B32, long long* rec0, long long* status, hipStream_t s);

// ansatz1.hip: per-node optimisation of B^* (FP64)
void launch_a1_bands(double2* out, int M, int nb, hipStream_t s);
void launch_a1_ones(double2* out, int64_t n, hipStream_t s);
void launch_a1_products(const double2* a, double2* prod, int Ms, int d0, int nd, int npair, double scale,
                        hipStream_t s);
void launch_a1_fold(const double2* R, const double2* h, double2* V, int M, int Ms, int nd, int npair, hipStream_t s);
void launch_a1_solve(const Geo& g, const NodesDev& nd, const double2* S, const double2* Ktab, int qK, double rho,
                     double2* B64, float2* B32, long long* status, hipStream_t s);

}  // namespace infft
