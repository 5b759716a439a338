// Oversampled FFT F / F^* of the NFFT (2.5): unnormalised, exponent sign +1 for F and -1 for F^*.
//
// One kernel launch computes `nseq` independent sub-transforms of length n, `rows` of them per
// workgroup, entirely in LDS with mixed-radix (2, 3, 4, 5, 7, 8) Stockham autosort stages.  A
// length that does not fit one workgroup is split four-step style (n = n1 n2, twiddle between
// the passes, applied at the first pass's store); 2-D grids transform rows then columns.  The
// first load and the last store of a transform carry the work around it:
//   LD_DECONV  zero-padding of the centred coefficients onto the M_sigma grid, scaled by D (2.4)
//   LD_HALO    the spread grid plus the halo strips its neighbouring tiles wrote
//   ST_DECONV  truncation to the centred M range and scaling by D^* (2.8)
#include "internal.hpp"

namespace infft {

// Complex elements per thread at most: a workgroup holds FFT_THREADS * E elements, 4096 (FP32) or
// 2048 (FP64).  512 threads with fewer elements each keep more loads of a pass in flight than 256
// threads with twice as many (1-D 2^17-point passes: step 0.149 -> 0.145 ms; 1024 threads were
// slower again).
constexpr int FFT_E32 = 8;
constexpr int FFT_E64 = 4;

size_t fft_lds_bytes(const FftPass& p, size_t csize) {
    return ((size_t)p.rows * (p.n + 1) + (size_t)p.n) * csize;
}

int fft_capacity(bool fp64) { return FFT_THREADS * (fp64 ? FFT_E64 : FFT_E32); }
// Batched FP32 passes of up to FFT_THREADS * FFT_EB32 elements per workgroup run in a kernel built
// for at most FFT_EB32 elements per thread: without the 8-element body it fits 80 VGPRs (six
// waves per SIMD), so three 512-thread workgroups share a CU instead of two (those passes 14-23 %
// faster per launch).
constexpr int FFT_EB32 = 4;
int fft_batched_small_capacity() { return FFT_THREADS * FFT_EB32; }

// ------------------------------------------------------------------ radix-r DFT, sign -1

template <typename C> __device__ inline C mul_mi(C a) {  // a * (-i)
    C r;
    r.x = a.y;
    r.y = -a.x;
    return r;
}

template <typename C, int RADIX> struct Dft;

template <typename C> struct Dft<C, 2> {
    __device__ static void run(C* v) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename C> struct Dft<C, 4> {
    __device__ static void run(C* v) {
        const C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const C t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <typename C> struct Dft<C, 8> {
    __device__ static void run(C* v) {
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<C, 4>::run(e);
        Dft<C, 4>::run(o);
        using R = decltype(v[0].x);
        const R h = (R)0.70710678118654752440;
        // o[k] * e^{-2 pi i k / 8}
        C o1, o3;
        o1.x = h * (o[1].x + o[1].y);
        o1.y = h * (o[1].y - o[1].x);
        const C o2 = mul_mi(o[2]);
        o3.x = h * (o[3].y - o[3].x);
        o3.y = -h * (o[3].x + o[3].y);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

// Odd radices: direct O(r^2) sum with W_r^j = cw[j] + i sw[j] = e^{-2 pi i j / r}
// (cos and sin of 2 pi j / r from their closed forms: sqrt(3)/2, (sqrt(5) -+ 1)/4, ...).
template <int RADIX> struct OddW;
template <> struct OddW<3> {
    static constexpr double c1 = -0.5, s1 = 0.86602540378443864676;
    __device__ static double c(int j) { return j == 0 ? 1.0 : c1; }
    __device__ static double s(int j) { return j == 0 ? 0.0 : (j == 1 ? -s1 : s1); }
};
template <> struct OddW<5> {
    static constexpr double c1 = 0.30901699437494742410, s1 = 0.95105651629515357212;
    static constexpr double c2 = -0.80901699437494742410, s2 = 0.58778525229247312917;
    __device__ static double c(int j) { return j == 0 ? 1.0 : (j == 1 || j == 4) ? c1 : c2; }
    __device__ static double s(int j) {
        return j == 0 ? 0.0 : j == 1 ? -s1 : j == 2 ? -s2 : j == 3 ? s2 : s1;
    }
};
template <> struct OddW<7> {
    static constexpr double c1 = 0.62348980185873353053, s1 = 0.78183148246802980871;
    static constexpr double c2 = -0.22252093395631440429, s2 = 0.97492791218182360702;
    static constexpr double c3 = -0.90096886790241912624, s3 = 0.43388373911755812048;
    __device__ static double c(int j) {
        return j == 0 ? 1.0 : (j == 1 || j == 6) ? c1 : (j == 2 || j == 5) ? c2 : c3;
    }
    __device__ static double s(int j) {
        return j == 0 ? 0.0 : j == 1 ? -s1 : j == 2 ? -s2 : j == 3 ? -s3 : j == 4 ? s3 : j == 5 ? s2 : s1;
    }
};

template <typename C, int RADIX> struct DftOdd {
    __device__ static void run(C* v) {
        using R = decltype(v[0].x);
        C out[RADIX];
#pragma unroll
        for (int q = 0; q < RADIX; ++q) {
            C acc = v[0];
#pragma unroll
            for (int p = 1; p < RADIX; ++p) {
                const int j = (p * q) % RADIX;
                const R cw = (R)OddW<RADIX>::c(j), sw = (R)OddW<RADIX>::s(j);
                acc.x += v[p].x * cw - v[p].y * sw;
                acc.y += v[p].x * sw + v[p].y * cw;
            }
            out[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < RADIX; ++q) v[q] = out[q];
    }
};
template <typename C> struct Dft<C, 3> : DftOdd<C, 3> {};
template <typename C> struct Dft<C, 5> : DftOdd<C, 5> {};
template <typename C> struct Dft<C, 7> : DftOdd<C, 7> {};

// ------------------------------------------------------------------ index division

// Division by a workgroup-uniform divisor d: a shift when d is a power of two (every length of a
// power-of-two grid, and the autotuned row counts).  Otherwise, with MD, the high half of x m with
// m = floor((2^32 - 1) / d) + 1, which is floor(x / d) whenever x d < 2^32 (with m d = 2^32 + e,
// 0 < e < d: x m / 2^32 = x / d + x e / (d 2^32), and x e < 2^32 keeps the fraction below 1), and
// the integer division where a dividend up to xmax could break that bound; without MD the integer
// division.  The tests are uniform, so only one path runs; m is kept in a scalar register.  MD
// serves the batched passes, whose lengths are rarely powers of two; the single-plan passes keep
// the plain form, whose registers stay within four waves per SIMD.
template <bool MD> struct UDiv {
    uint32_t d, m;
    int sh;
    bool p2, mul;
    __device__ UDiv(uint32_t dv, uint32_t xmax) : d(dv), sh(__builtin_ctz(dv)), p2((dv & (dv - 1)) == 0) {
        if (MD) {
            m = (uint32_t)__builtin_amdgcn_readfirstlane((int)(0xFFFFFFFFu / dv + 1u));
            mul = (uint64_t)xmax * dv < (1ull << 32);
        } else {
            m = 0;
            mul = false;
        }
    }
    __device__ uint32_t div(uint32_t x) const {
        if (MD) return p2 ? (x >> sh) : mul ? __umulhi(x, m) : x / d;
        return p2 ? (x >> sh) : x / d;
    }
    __device__ uint32_t mod(uint32_t x) const {
        if (MD) return x - div(x) * d;
        return p2 ? (x & (d - 1)) : x - (x / d) * d;
    }
};

// ------------------------------------------------------------------ one Stockham stage in LDS

template <typename R, int RADIX, int E, int MD>
__device__ inline void stage(cx<R>* lds, int ld, int rows, int n, int Ns, int sign,
                             const cx<R>* __restrict__ tw) {
    using C = cx<R>;
    constexpr int CM = (E + RADIX - 1) / RADIX;
    const int nbr = n / RADIX;
    const int nb = rows * nbr;
    // dividends: b < nb and j < nbr
    const UDiv<(MD != 0)> dnbr((uint32_t)nbr, (uint32_t)nb), dNs((uint32_t)Ns, (uint32_t)nbr);
    C v[CM][RADIX];
#pragma unroll
    for (int ci = 0; ci < CM; ++ci) {
        const int b = threadIdx.x + ci * FFT_THREADS;
        if (b < nb) {
            const int row = (int)dnbr.div((uint32_t)b), j = b - row * nbr;
#pragma unroll
            for (int q = 0; q < RADIX; ++q) v[ci][q] = lds[row * ld + j + q * nbr];
        }
    }
    __syncthreads();
    const int tstride = n / (Ns * RADIX);
#pragma unroll
    for (int ci = 0; ci < CM; ++ci) {
        const int b = threadIdx.x + ci * FFT_THREADS;
        if (b < nb) {
            const int row = (int)dnbr.div((uint32_t)b), j = b - row * nbr;
            const int jm = (int)dNs.mod((uint32_t)j);
#pragma unroll
            for (int q = 1; q < RADIX; ++q) {
                C w = tw[q * jm * tstride];
                if (sign > 0) w.y = -w.y;
                v[ci][q] = cmul(v[ci][q], w);
            }
            if (sign > 0) {
#pragma unroll
                for (int q = 0; q < RADIX; ++q) v[ci][q].y = -v[ci][q].y;
            }
            Dft<C, RADIX>::run(v[ci]);
            if (sign > 0) {
#pragma unroll
                for (int q = 0; q < RADIX; ++q) v[ci][q].y = -v[ci][q].y;
            }
            const int idxD = (j - jm) * RADIX + jm;
#pragma unroll
            for (int q = 0; q < RADIX; ++q) lds[row * ld + idxD + q * Ns] = v[ci][q];
        }
    }
    __syncthreads();
}

template <typename R, int E, int MD>
__device__ inline void lds_fft(cx<R>* lds, int ld, int rows, const FftPass& P, const cx<R>* tw) {
    int Ns = 1;
    for (int s = 0; s < P.nst; ++s) {
        const int r = P.rad[s];
        switch (r) {
            case 2: stage<R, 2, E, MD>(lds, ld, rows, P.n, Ns, P.sign, tw); break;
            case 3: stage<R, 3, E, MD>(lds, ld, rows, P.n, Ns, P.sign, tw); break;
            case 4: stage<R, 4, E, MD>(lds, ld, rows, P.n, Ns, P.sign, tw); break;
            case 5: stage<R, 5, E, MD>(lds, ld, rows, P.n, Ns, P.sign, tw); break;
            case 7: stage<R, 7, E, MD>(lds, ld, rows, P.n, Ns, P.sign, tw); break;
            default: stage<R, 8, E, MD>(lds, ld, rows, P.n, Ns, P.sign, tw); break;
        }
        Ns *= r;
    }
}

// ------------------------------------------------------------------ fused loads / stores

// centred coefficient index of grid position p (or -1 when the frequency is outside the M range)
__device__ inline int coeff_index(int p, int Ms, int M) {
    const int k = (p < Ms / 2) ? p : p - Ms;
    return (k >= -M / 2 && k < M / 2) ? k + M / 2 : -1;
}

// Grid position -> (row, column) of a D-dimensional grid (D = 1: the position itself).
template <int D> __device__ inline void grid_rc(const Geo& g, int64_t pos, int& p0, int& p1) {
    if (D == 1) {
        p0 = (int)pos;
        p1 = 0;
    } else {
        p0 = (int)(pos / g.Ms[1]);
        p1 = (int)(pos - (int64_t)p0 * g.Ms[1]);
    }
}

// The element loads are branch-free where the pass is one-dimensional (a coefficient outside the
// M range is loaded at index 0 and replaced by zero), so that the loads of a thread's elements
// can all be in flight together.
template <typename R, int LD, int D>
__device__ inline cx<R> load_elem(const FftIO& io, const FftPass& P, const Geo& g, int64_t r, int64_t pos) {
    using C = cx<R>;
    if (LD == LD_GRID) {
        return ((const C*)io.in)[r * P.in_rs + pos];
    } else if (LD == LD_DECONV) {
        int p0, p1;
        grid_rc<D>(g, pos, p0, p1);
        const int i0 = coeff_index(p0, g.Ms[0], g.M[0]);
        const int i1 = (D == 1) ? 0 : coeff_index(p1, g.Ms[1], g.M[1]);
        const bool ok = i0 >= 0 && i1 >= 0;
        const int j0 = max(i0, 0), j1 = max(i1, 0);
        R s = ((const R*)io.D0)[j0];
        if (D == 2) s *= ((const R*)io.D1)[j1];
        const C v = ((const C*)io.in)[r * P.in_rs + (int64_t)j0 * g.M[1] + j1];
        return ok ? cscale(v, s) : cmake((R)0, (R)0);
    } else {  // LD_HALO
        C v = ((const C*)io.in)[r * P.in_rs + pos];
        const int w2 = 2 * g.m;
        int p0, p1;
        grid_rc<D>(g, pos, p0, p1);
        const int t0 = p0 / g.TS[0], o0 = p0 - t0 * g.TS[0];
        const int t1 = p1 / g.TS[1], o1 = p1 - t1 * g.TS[1];
        const int tm0 = (t0 == 0) ? g.ntile[0] - 1 : t0 - 1;
        const int tm1 = (t1 == 0) ? g.ntile[1] - 1 : t1 - 1;
        if (o0 < w2) {
            const int64_t tile = (int64_t)tm0 * g.ntile[1] + t1;
            v = cadd(v, ((const C*)io.h0)[r * io.halo_rs0 + (tile * w2 + o0) * g.TS[1] + o1]);
        }
        if (D == 2 && o1 < w2) {
            const int64_t tile = (int64_t)t0 * g.ntile[1] + tm1;
            v = cadd(v, ((const C*)io.h1)[r * io.halo_rs1 + (tile * g.TS[0] + o0) * w2 + o1]);
            if (o0 < w2) {
                const int64_t tc = (int64_t)tm0 * g.ntile[1] + tm1;
                v = cadd(v, ((const C*)io.h01)[r * io.halo_rs01 + (tc * w2 + o0) * w2 + o1]);
            }
        }
        return v;
    }
}

// What a store needs from memory besides the transformed value, loaded with the pass's input:
// the two table entries of the inter-pass twiddle (ST_TWIDDLE) or the deconvolution factor
// (ST_DECONV).
template <typename R> struct StoreOperand {
    cx<R> hi, lo;
    R scale;
};

template <typename R, int ST, int D>
__device__ inline void store_prefetch(const FftIO& io, const FftPass& P, const Geo& g, int64_t pos, int64_t q,
                                      int k, StoreOperand<R>& o) {
    using C = cx<R>;
    if (ST == ST_TWIDDLE) {
        // q < n2 and k < n1, so e = q k < N: no reduction; twB is a power of two
        const uint32_t e = (uint32_t)q * (uint32_t)k;
        o.hi = ((const C*)P.twHi)[e >> P.twShift];
        o.lo = ((const C*)P.twLo)[e & (uint32_t)(P.twB - 1)];
    } else if (ST == ST_DECONV) {
        int p0, p1;
        grid_rc<D>(g, pos, p0, p1);
        const int i0 = coeff_index(p0, g.Ms[0], g.M[0]);
        const int i1 = (D == 1) ? 0 : coeff_index(p1, g.Ms[1], g.M[1]);
        o.scale = ((const R*)io.D0)[max(i0, 0)];
        if (D == 2) o.scale *= ((const R*)io.D1)[max(i1, 0)];
    }
}

template <typename R, int ST, int D>
__device__ inline void store_elem(const FftIO& io, const FftPass& P, const Geo& g, int64_t r, int64_t pos,
                                  const StoreOperand<R>& o, cx<R> v) {
    using C = cx<R>;
    if (ST == ST_GRID) {
        ((C*)io.out)[r * P.out_rs + pos] = v;
    } else if (ST == ST_TWIDDLE) {
        C w = cmul(o.hi, o.lo);
        if (P.sign > 0) w.y = -w.y;
        ((C*)io.out)[r * P.out_rs + pos] = cmul(v, w);
    } else {  // ST_DECONV: truncation to the M range
        int p0, p1;
        grid_rc<D>(g, pos, p0, p1);
        const int i0 = coeff_index(p0, g.Ms[0], g.M[0]);
        const int i1 = (D == 1) ? 0 : coeff_index(p1, g.Ms[1], g.M[1]);
        if (i0 < 0 || i1 < 0) return;
        ((C*)io.out)[r * P.out_rs + (int64_t)i0 * g.M[1] + i1] = cscale(v, o.scale);
    }
}

// One workgroup's share of a pass: sub-transforms blk * rows .. of the pass.  A pass moves little
// data per workgroup (a few elements per thread), so its time is memory latency: every global
// load of the workgroup (the elements, the stage twiddle table, the store operands) is issued
// before the first is used, and the pass waits on memory once instead of once per element.
template <typename R, int E, int LD, int ST, int D, int MD>
__device__ inline void fft_block(const FftPass& P, int64_t nseq, const FftIO& io, const Geo& g, int64_t blk) {
    using C = cx<R>;
    extern __shared__ char smem_raw[];
    C* lds = (C*)smem_raw;
    const int ld = P.n + 1;
    const int64_t seq0 = blk * (int64_t)P.rows;
    if (seq0 >= nseq) return;
    const int rows = (int)min((int64_t)P.rows, nseq - seq0);
    const int tot = rows * P.n;   // at most FFT_THREADS * E
    // dividends: element indices below tot, sequence indices below nseq
    const UDiv<(MD != 0)> drows((uint32_t)rows, (uint32_t)tot), dn((uint32_t)P.n, (uint32_t)tot),
        dnq((uint32_t)P.nq, (uint32_t)min(nseq, (int64_t)0xFFFFFFFF));
    // the stage twiddle table follows the data in LDS
    C* s_tw = lds + (int64_t)P.rows * ld;
    const C* gtw = (const C*)P.tw;
    // Every load runs unconditionally, at an index clamped into range: a thread past the end
    // re-reads the last element (or table entry) and writes it to the same LDS slot as its owner,
    // with the same value.  Without branches the unrolled loops are straight-line code and the
    // loads are issued back to back.
    C dat[E], twt[E];
    StoreOperand<R> so[(ST == ST_GRID) ? 1 : E];
    int slot[E];
#pragma unroll
    for (int it = 0; it < E; ++it) {
        const int L = threadIdx.x + it * FFT_THREADS;
        twt[it] = gtw[min(L, P.n - 1)];
        const int Lc = min(L, tot - 1);
        int row, i;
        if (P.in_rowfast) { i = (int)drows.div((uint32_t)Lc); row = Lc - i * rows; }
        else { row = (int)dn.div((uint32_t)Lc); i = Lc - row * P.n; }
        slot[it] = row * ld + i;
        const uint32_t s = (uint32_t)(seq0 + row);
        const uint32_t r = dnq.div(s), q = s - r * (uint32_t)P.nq;
        dat[it] = load_elem<R, LD, D>(io, P, g, r, (int64_t)q * P.in_qs + (int64_t)i * P.in_is);
        if (ST != ST_GRID) {
            int orow, k;
            if (P.out_rowfast) { k = (int)drows.div((uint32_t)Lc); orow = Lc - k * rows; }
            else { orow = (int)dn.div((uint32_t)Lc); k = Lc - orow * P.n; }
            const uint32_t os = (uint32_t)(seq0 + orow);
            const uint32_t oq = os - dnq.div(os) * (uint32_t)P.nq;
            store_prefetch<R, ST, D>(io, P, g, (int64_t)oq * P.out_qs + (int64_t)k * P.out_ks, oq, k, so[it]);
        }
    }
#pragma unroll
    for (int it = 0; it < E; ++it) {
        s_tw[min((int)threadIdx.x + it * FFT_THREADS, P.n - 1)] = twt[it];
        lds[slot[it]] = dat[it];
    }
    __syncthreads();
    lds_fft<R, E, MD>(lds, ld, rows, P, s_tw);
#pragma unroll
    for (int it = 0; it < E; ++it) {
        const int L = threadIdx.x + it * FFT_THREADS;
        if (L < tot) {
            int row, k;
            if (P.out_rowfast) { k = (int)drows.div((uint32_t)L); row = L - k * rows; }
            else { row = (int)dn.div((uint32_t)L); k = L - row * P.n; }
            const uint32_t s = (uint32_t)(seq0 + row);
            const uint32_t r = dnq.div(s), q = s - r * (uint32_t)P.nq;
            store_elem<R, ST, D>(io, P, g, r, (int64_t)q * P.out_qs + (int64_t)k * P.out_ks,
                                 so[(ST == ST_GRID) ? 0 : it], lds[row * ld + k]);
        }
    }
}

// The body is instantiated for the elements per thread the pass needs (a power of two up to the
// capacity E), so no thread loads more than one element past the end; the choice and the
// dimension are uniform branches at the kernel's entry.
template <typename R, int E, int LD, int ST, int D, int MD>
__device__ inline void fft_block_e(const FftPass& P, int64_t nseq, const FftIO& io, const Geo& g, int64_t blk) {
    const int ept = (P.rows * P.n + FFT_THREADS - 1) / FFT_THREADS;
    if (ept <= 1) fft_block<R, 1, LD, ST, D, MD>(P, nseq, io, g, blk);
    else if (ept <= 2) fft_block<R, 2, LD, ST, D, MD>(P, nseq, io, g, blk);
    else if (ept <= 4) fft_block<R, 4, LD, ST, D, MD>(P, nseq, io, g, blk);
    else if (E <= 8 || ept <= 8) fft_block<R, (E < 8 ? E : 8), LD, ST, D, MD>(P, nseq, io, g, blk);
    else fft_block<R, E, LD, ST, D, MD>(P, nseq, io, g, blk);
}

template <typename R, int E, int LD, int ST>
__device__ inline void fft_block_d(const FftPass& P, int64_t nseq, const FftIO& io, const Geo& g, int64_t blk) {
    if (g.d == 1) fft_block_e<R, E, LD, ST, 1, 0>(P, nseq, io, g, blk);
    else fft_block_e<R, E, LD, ST, 2, 0>(P, nseq, io, g, blk);
}

template <typename R, int E, int LD, int ST>
__global__ void __launch_bounds__(FFT_THREADS) k_fft(FftPass P, FftIO io, Geo g) {
    fft_block_d<R, E, LD, ST>(P, P.nseq, io, g, xcd_block(blockIdx.x, gridDim.x));
}

// Passes of many problems in one launch: workgroup -> (job, block of that job's pass).  A job's
// caller-side array is the batch array plus nrhs times the job's offset (problem-major layout);
// its sub-transform count follows the call's nrhs, so blocks planned for more right-hand sides
// find no work and return.
// MD: 1 for the batched kernel, 2 for the small one, so that each kernel has its own (inlined)
// copies of the pass body and the small kernel's register bound applies to all of it
template <typename R, int E, int LD, int ST, int MD>
__device__ __forceinline__ void fft_batched_body(const FftJob* __restrict__ jobs, const int2* __restrict__ bmap,
                                        const void* user_in, void* user_out, int nrhs) {
    const int2 b = bmap[xcd_block(blockIdx.x, gridDim.x)];
    const FftJob& J = jobs[b.x];
    // the pass is read in place (a local copy would put its radix table, indexed per stage, in
    // scratch); only the sequence count follows the call's nrhs
    FftIO io = J.io;
    if (J.user_in) io.in = (const cx<R>*)user_in + (int64_t)nrhs * J.user_off;
    if (J.user_out) io.out = (cx<R>*)user_out + (int64_t)nrhs * J.user_off;
    fft_block_e<R, E, LD, ST, 1, MD>(J.pass, J.pass.nq * nrhs, io, J.g, b.y);   // batches are 1-D
}

template <typename R, int E, int LD, int ST>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_batched(const FftJob* __restrict__ jobs,
                                                             const int2* __restrict__ bmap, const void* user_in,
                                                             void* user_out, int nrhs) {
    fft_batched_body<R, E, LD, ST, 1>(jobs, bmap, user_in, user_out, nrhs);
}

// FP32 passes of at most fft_batched_small_capacity() elements per workgroup (six waves per SIMD)
template <int LD, int ST>
__global__ void __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(6)))
k_fft_batched_small(const FftJob* __restrict__ jobs, const int2* __restrict__ bmap, const void* user_in,
                    void* user_out, int nrhs) {
    fft_batched_body<float, FFT_EB32, LD, ST, 2>(jobs, bmap, user_in, user_out, nrhs);
}

template <typename R>
void launch_fft_pass(const FftPass& p, const FftIO& io, const Geo& g, int ld, int st, hipStream_t s) {
    constexpr int E = (sizeof(R) == 8) ? FFT_E64 : FFT_E32;
    const unsigned blocks = (unsigned)((p.nseq + p.rows - 1) / p.rows);
    const size_t shm = fft_lds_bytes(p, sizeof(cx<R>));
#define INFFT_FFT_CASE(L_, S_)                                                                  \
    if (ld == L_ && st == S_) {                                                                 \
        hipLaunchKernelGGL((k_fft<R, E, L_, S_>), dim3(blocks), dim3(FFT_THREADS), shm, s, p, io, g); \
        return;                                                                                 \
    }
    INFFT_FFT_CASE(LD_GRID, ST_GRID)
    INFFT_FFT_CASE(LD_GRID, ST_TWIDDLE)
    INFFT_FFT_CASE(LD_GRID, ST_DECONV)
    INFFT_FFT_CASE(LD_DECONV, ST_GRID)
    INFFT_FFT_CASE(LD_DECONV, ST_TWIDDLE)
    INFFT_FFT_CASE(LD_HALO, ST_GRID)
    INFFT_FFT_CASE(LD_HALO, ST_TWIDDLE)
    INFFT_FFT_CASE(LD_HALO, ST_DECONV)
    INFFT_FFT_CASE(LD_DECONV, ST_DECONV)
#undef INFFT_FFT_CASE
}

template void launch_fft_pass<float>(const FftPass&, const FftIO&, const Geo&, int, int, hipStream_t);
template void launch_fft_pass<double>(const FftPass&, const FftIO&, const Geo&, int, int, hipStream_t);

template <typename R>
void launch_fft_batched(const FftJob* jobs, const int2* bmap, int nblocks, size_t shm, int ld, int st,
                        const void* user_in, void* user_out, int nrhs, bool small, hipStream_t s) {
    if (nblocks <= 0) return;
    constexpr int E = (sizeof(R) == 8) ? FFT_E64 : FFT_E32;
#define INFFT_FFTB_CASE(L_, S_)                                                                       \
    if (ld == L_ && st == S_) {                                                                       \
        if (small && sizeof(R) == 4)                                                                  \
            hipLaunchKernelGGL((k_fft_batched_small<L_, S_>), dim3(nblocks), dim3(FFT_THREADS), shm, s, \
                               jobs, bmap, user_in, user_out, nrhs);                                  \
        else                                                                                          \
            hipLaunchKernelGGL((k_fft_batched<R, E, L_, S_>), dim3(nblocks), dim3(FFT_THREADS), shm, s,  \
                               jobs, bmap, user_in, user_out, nrhs);                                  \
        return;                                                                                       \
    }
    INFFT_FFTB_CASE(LD_DECONV, ST_GRID)
    INFFT_FFTB_CASE(LD_DECONV, ST_TWIDDLE)
    INFFT_FFTB_CASE(LD_GRID, ST_GRID)
    INFFT_FFTB_CASE(LD_GRID, ST_TWIDDLE)
    INFFT_FFTB_CASE(LD_GRID, ST_DECONV)
#undef INFFT_FFTB_CASE
}

template void launch_fft_batched<float>(const FftJob*, const int2*, int, size_t, int, int, const void*, void*, int,
                                        bool, hipStream_t);
template void launch_fft_batched<double>(const FftJob*, const int2*, int, size_t, int, int, const void*, void*,
                                         int, bool, hipStream_t);

}  // namespace infft
