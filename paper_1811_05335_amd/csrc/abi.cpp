// C ABI of libinfft: argument validation, the plan (geometry, device workspace, FFT schedule)
// and the order of kernel launches for each entry point declared in include/infft.h.
#include "infft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace infft;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(INFFT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK()                                                                     \
    do {                                                                                   \
        hipError_t e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess) return fail(INFFT_EDEVICE, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

// radices the LDS Stockham kernel implements, largest first
bool factor_radices(int n, std::vector<int>& rad) {
    rad.clear();
    for (int r : {8, 4, 2}) {
        while (n % r == 0 && n > 1) {
            rad.push_back(r);
            n /= r;
        }
    }
    for (int r : {7, 5, 3}) {
        while (n % r == 0) {
            rad.push_back(r);
            n /= r;
        }
    }
    return n == 1 && (int)rad.size() <= FFT_MAX_STAGES;
}

struct TwTable {
    int64_t n = 0;
    double2* t64 = nullptr;
    float2* t32 = nullptr;
};

struct FftStep {
    FftPass pass;
    int ld, st;
    int in_buf, out_buf;   // 0 = caller's array, 1 = grid, 2 = scratch grid
};

}  // namespace

struct BatchState;
void batch_free(BatchState* b);

// One batch of a recorded large-problem pass: its problems (a range of the record's descriptors,
// sorted by size, largest first) and the task segments of its launches.
struct BigBatch {
    int np = 0;
    int T0 = 0;                  // block columns of its largest problem
    int64_t prob_off = 0;
    std::vector<int> nblk;       // block columns per problem
    std::vector<int64_t> seg;    // Gram tiles, then per block column the panel and trailing tiles
    std::vector<int64_t> fseg;   // forward substitution per block step
    std::vector<int64_t> bseg;   // backward substitution per block step
};

// A recorded large-problem pass: built outside graph capture, replayed under capture.
struct BigSched {
    bool built = false;
    int count = 0;
    int nmin = 0, nmax = 0;
    std::vector<BigBatch> batches;
    BigProb* probs = nullptr;    // descriptors of all batches
    int4* tasks = nullptr;       // task lists of all batches
    int* fail = nullptr;         // per problem: non-positive pivot
    int* slot = nullptr;         // per grid index: its problem in the record, -1 otherwise
    int* flag = nullptr;         // [0] set when the listed problems differ from the record;
                                 // [1] the generation of the current record
    int gen = 0;
    int64_t probs_cap = 0, tasks_cap = 0, fail_cap = 0;
};

// alignment of every buffer carved from a workspace (and of the workspace itself)
constexpr int WS_ALIGN = 256;

struct infft_plan_s {
    Geo g{};
    int prec = INFFT_F64;
    int max_rhs = 1;
    double rho = 1e-8;
    double sigma = 2.0;
    hipStream_t stream = nullptr;
    int device = -1;   // the device current when the plan was made
    std::vector<void*> allocs;
    int64_t bytes = 0;
    // workspace plans carve every buffer from the caller's workspace (ws_base, ws_size); a
    // measuring plan only counts the bytes (no device memory, no device work)
    bool ws_mode = false;
    bool measure = false;
    char* ws_base = nullptr;
    size_t ws_size = 0;
    size_t ws_used = 0;

    NodesDev nd{};
    int* counts = nullptr;
    int* nonfinite = nullptr;     // per-workgroup non-finite node counts of the preprocessing
    bool nodes_zeroed = false;    // counters and fill cursors are zero (after the first reset)
    int* fill = nullptr;
    int* bsum = nullptr;
    long long* status = nullptr;

    double* D64[MAX_D] = {nullptr, nullptr};
    float* D32[MAX_D] = {nullptr, nullptr};
    // factors of the inverse (B optimisation, modified adjoint and its adjoint): the same as D,
    // or for the Dirichlet kernel of Remark 3.19 1/M_sigma with the entry of k = -M/2 zero
    int inv_kernel = INFFT_KERNEL_WINDOW;
    double* Di64[MAX_D] = {nullptr, nullptr};
    float* Di32[MAX_D] = {nullptr, nullptr};
    double2* Ktab[MAX_D] = {nullptr, nullptr};
    double2* Qtab[MAX_D] = {nullptr, nullptr};
    double* Kstab = nullptr;   // 1-D symmetric (real) parts of K and Q
    double* Qstab = nullptr;
    double dM = 0.0;
    int qK = 0, qQ = 0;
    double lam = 0.0;

    std::vector<long double> wpoly_host;   // window polynomial coefficients, uploaded at set-up
    void* tune_buf = nullptr;              // coefficient buffer of the autotuner
    // workspace plans: memory for local problems beyond the register tiers, and the work arrays and
    // inner-plan workspaces of Algorithm 3.10 (when the plan was made with ansatz1)
    char* large_arena = nullptr;
    int64_t large_arena_bytes = 0;
    void* a1_ws[2] = {nullptr, nullptr};
    size_t a1_ws_bytes[2] = {0, 0};
    std::vector<TwTable> tw;
    TwTable split_lo, split_hi;
    std::vector<FftStep> to_grid;    // coefficients -> grid (sign +1, with D)
    std::vector<FftStep> to_coeff;   // grid + halos -> coefficients (sign -1, with D^*)

    void* grid = nullptr;      // the work buffers of the current slot
    void* grid2 = nullptr;
    void* h0 = nullptr;
    void* h1 = nullptr;
    void* h01 = nullptr;
    struct Slot {
        void *grid, *grid2, *h0, *h1, *h01;
        int trafo_rhs = 0;   // > 0: grid holds F D fhat of the last nfft_trafo (that many RHS)
    };
    std::vector<Slot> slots;   // work_slots sets of the five buffers above
    int cur_slot = 0;
    int64_t hrs0 = 0, hrs1 = 0, hrs01 = 0;
    SpreadWork spwork{};            // 2-D: work list of the tiled spreading (rebuilt by set_nodes)
    int* sp_offs = nullptr;
    int* sp_bsum = nullptr;
    int rchunk = 1;
    // FFT workgroups a pass should at least have before sub-transforms are packed together
    // (a batch plan's problems share their launches, so they pack as many as fit)
    int64_t fft_min_blocks = 1024;
    // rows per FFT workgroup chosen by infft_autotune, per step of each direction (0: default)
    int fft_rows[2][2] = {{0, 0}, {0, 0}};

    // B_opt in sorted order.  FP64 plans keep B64 only; FP32 plans apply B32, and their B
    // optimisation writes B32 alone: the FP64 values (infft_get_B, export, the node gradient
    // through B_opt(x)) are recomputed into B64 on demand.  Algorithm 3.10 and an import write both.
    double2* B64 = nullptr;
    float2* B32 = nullptr;
    // the copies the tiers of the current B optimisation write (the large-problem pass reads them)
    double2* out_B64 = nullptr;
    float2* out_B32 = nullptr;
    int bopt_kind = 0;         // what B holds: 0 B_opt of Algorithm 3.17, 1 B_opt^* of Algorithm 3.10
    // Algorithm 3.10: inner FP64 plans and work arrays, made on first use
    infft_plan_s* a1_pplan = nullptr;   // bandwidth 2M, sigma 2: the Toeplitz symbol P(q)
    infft_plan_s* a1_fplan = nullptr;   // FP64 twin of an FP32 plan: length-M_sigma FFTs in FP64
    double2* a1_buf = nullptr;
    int64_t a1_cap = 0;
    bool a1_R_ready = false;            // the node-independent correlations R_d are in a1_buf
    int* lists = nullptr;      // one list of grid indices for problems passed to the wider tier
    int* lcount = nullptr;
    long long* stat_rec = nullptr;   // per-block statistics of the solve kernels
    int stat_nrec = 0;
    bool bopt_ready = false;

    // many 1-D problems in one plan (nullptr for a single problem)
    struct BatchState* batch = nullptr;

    // large local problems: sizes, one batch of matrices and members (allocated when first
    // needed and grown on demand, or placed in a workspace plan's workspace), and the records of
    // the pass (0: the precompute, 1: the node gradient through B_opt(x))
    int* big_n = nullptr;
    BigSched big_sched[2];
    double2* big_A = nullptr;
    int64_t big_A_cap = 0;
    int* big_midx = nullptr;
    int* big_mtap = nullptr;
    double2* big_mz = nullptr;
    double2* big_mr = nullptr;
    double2* big_mb = nullptr;
    int64_t big_m_cap = 0;

    // optional event timing of one kernel class
    int prof_class = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;

    size_t csize() const { return prec == INFFT_F32 ? sizeof(float2) : sizeof(double2); }
    int taps() const { return g.d == 1 ? 2 * g.m + 1 : (2 * g.m + 1) * (2 * g.m + 1); }

    template <typename T>
    int alloc(T** p, int64_t count) {
        void* q = nullptr;
        const size_t nb = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        if (ws_mode) {
            const size_t off = (ws_used + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
            if (off + nb > ws_size || off + nb < off)
                return fail(INFFT_ENOMEM, "workspace of %zu bytes exhausted (%zu more needed)", ws_size, off + nb - ws_size);
            ws_used = off + nb;
            bytes += (int64_t)nb;
            // a measuring plan hands out addresses that are never used
            *p = (T*)((measure ? (char*)(uintptr_t)WS_ALIGN : ws_base) + off);
            return INFFT_OK;
        }
        hipError_t e = hipMalloc(&q, nb);
        if (e != hipSuccess) return fail(INFFT_ENOMEM, "hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
        allocs.push_back(q);
        bytes += (int64_t)nb;
        *p = (T*)q;
        return INFFT_OK;
    }

    // Replaces *p by an allocation of at least `need` elements when it holds fewer.
    template <typename T>
    int grow(T** p, int64_t& cap, int64_t need) {
        if (need <= cap) return INFFT_OK;
        if (ws_mode)   // workspace plans place everything at plan time
            return fail(INFFT_ENOMEM, "workspace plan: %lld elements needed where %lld were placed",
                        (long long)need, (long long)cap);
        if (*p) {
            auto it = std::find(allocs.begin(), allocs.end(), (void*)*p);
            if (it != allocs.end()) allocs.erase(it);
            (void)hipFree(*p);
            bytes -= cap * (int64_t)sizeof(T);
            *p = nullptr;
            cap = 0;
        }
        const int64_t n = need + need / 4;
        int rc = alloc(p, n);
        if (rc) return rc;
        cap = n;
        return INFFT_OK;
    }

    // As grow, but the replaced allocation is kept until the plan is destroyed: graphs captured
    // earlier may still hold its address (their kernels return at once, yet read it in bounds).
    template <typename T>
    int grow_retire(T** p, int64_t& cap, int64_t need) {
        if (need <= cap) return INFFT_OK;
        if (ws_mode) return grow(p, cap, need);
        *p = nullptr;   // the old block stays in `allocs`, freed with the plan
        cap = 0;
        const int64_t n = need + need / 4;
        int rc = alloc(p, n);
        if (rc) return rc;
        cap = n;
        return INFFT_OK;
    }

    ~infft_plan_s() {
        if (batch) batch_free(batch);
        delete a1_pplan;
        delete a1_fplan;
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        if (!ws_mode)
            for (void* p : allocs) (void)hipFree(p);
    }
};

namespace {

// Brackets the launches between construction and destruction with two events when the plan
// times this kernel class.
struct ProfScope {
    infft_plan_s* P;
    bool on;
    ProfScope(infft_plan_s* p, int cls) : P(p), on(p->prof_class == cls) {
        if (on) record();
    }
    ~ProfScope() {
        if (on) record();
    }
    void record() {
        if (P->ev_used == P->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                on = false;
                return;
            }
            P->ev_pool.push_back(e);
        }
        (void)hipEventRecord(P->ev_pool[P->ev_used++], P->stream);
    }
};

const TwTable* find_tw(const infft_plan_s* P, int64_t n) {
    for (const TwTable& t : P->tw)
        if (t.n == n) return &t;
    return nullptr;
}

// Places the twiddle table of sub-length n (filled at plan set-up).
int reserve_tw(infft_plan_s* P, int64_t n) {
    if (find_tw(P, n)) return INFFT_OK;
    TwTable t;
    t.n = n;
    int rc = P->alloc(&t.t64, n);
    if (rc) return rc;
    if (P->prec == INFFT_F32 && (rc = P->alloc(&t.t32, n))) return rc;
    P->tw.push_back(t);
    return INFFT_OK;
}

const void* tw_ptr(const infft_plan_s* P, int64_t n) {
    const TwTable* t = find_tw(P, n);
    return P->prec == INFFT_F32 ? (const void*)t->t32 : (const void*)t->t64;
}

int choose_rows(int64_t n, int64_t nseq, int cap, int64_t min_blocks) {
    int64_t rows = std::max<int64_t>(1, nseq / min_blocks);
    rows = std::min<int64_t>(rows, cap / n);
    rows = std::min<int64_t>(rows, 16);
    return (int)std::max<int64_t>(rows, 1);
}

void fill_radices(FftPass& p) {
    std::vector<int> rad;
    factor_radices(p.n, rad);
    p.nst = (int)rad.size();
    for (int i = 0; i < p.nst; ++i) p.rad[i] = rad[i];
}

// Builds the two transform schedules for `nrhs` right-hand sides.
int build_schedule(infft_plan_s* P, int nrhs, std::vector<FftStep>& to_grid, std::vector<FftStep>& to_coeff) {
    const Geo& g = P->g;
    const int cap = fft_capacity(P->prec == INFFT_F64);
    to_grid.clear();
    to_coeff.clear();
    auto base = [&](int64_t n, int64_t nq) {
        FftStep s{};
        std::memset(&s.pass, 0, sizeof(s.pass));
        s.pass.n = (int)n;
        s.pass.nq = nq;
        s.pass.nseq = nq * nrhs;
        s.pass.rows = choose_rows(n, s.pass.nseq, cap, P->fft_min_blocks);
        s.pass.tw = tw_ptr(P, n);
        fill_radices(s.pass);
        return s;
    };
    if (g.d == 1 && g.Ms[0] <= cap) {
        FftStep s = base(g.Ms[0], 1);
        s.pass.in_is = 1;
        s.pass.out_ks = 1;
        FftStep a = s, b = s;
        a.pass.sign = +1; a.ld = LD_DECONV; a.st = ST_GRID; a.in_buf = 0; a.out_buf = 1;
        a.pass.in_rs = g.P; a.pass.out_rs = g.G;
        b.pass.sign = -1; b.ld = LD_GRID; b.st = ST_DECONV; b.in_buf = 1; b.out_buf = 0;  // 1-D: gather, no halos
        b.pass.in_rs = g.G; b.pass.out_rs = g.P;
        to_grid.push_back(a);
        to_coeff.push_back(b);
    } else if (g.d == 1) {
        // four-step split n = n1 * n2 chosen at plan time (n1 kept in split_hi.n)
        const int64_t n1 = P->split_hi.n;     // sub-length of the first pass
        const int64_t n2 = g.Ms[0] / n1;
        FftStep A = base(n1, n2), B = base(n2, n1);
        A.pass.in_qs = 1; A.pass.in_is = n2; A.pass.in_rowfast = 1;
        A.pass.out_qs = 1; A.pass.out_ks = n2; A.pass.out_rowfast = 1; A.pass.out_rs = g.G;
        A.pass.twN = g.Ms[0]; A.pass.twB = (int)P->split_lo.n;
        A.pass.twShift = 0;
        while ((1 << A.pass.twShift) < A.pass.twB) ++A.pass.twShift;
        A.pass.twLo = P->prec == INFFT_F32 ? (const void*)P->split_lo.t32 : (const void*)P->split_lo.t64;
        A.pass.twHi = P->prec == INFFT_F32 ? (const void*)P->split_hi.t32 : (const void*)P->split_hi.t64;
        B.pass.in_qs = n2; B.pass.in_is = 1; B.pass.in_rowfast = 0; B.pass.in_rs = g.G;
        B.pass.out_qs = 1; B.pass.out_ks = n1; B.pass.out_rowfast = 1;
        FftStep a1 = A, a2 = B, b1 = A, b2 = B;
        a1.pass.sign = +1; a1.ld = LD_DECONV; a1.st = ST_TWIDDLE; a1.in_buf = 0; a1.out_buf = 2; a1.pass.in_rs = g.P;
        a2.pass.sign = +1; a2.ld = LD_GRID; a2.st = ST_GRID; a2.in_buf = 2; a2.out_buf = 1; a2.pass.out_rs = g.G;
        b1.pass.sign = -1; b1.ld = LD_GRID; b1.st = ST_TWIDDLE; b1.in_buf = 1; b1.out_buf = 2; b1.pass.in_rs = g.G;
        b2.pass.sign = -1; b2.ld = LD_GRID; b2.st = ST_DECONV; b2.in_buf = 2; b2.out_buf = 0; b2.pass.out_rs = g.P;
        to_grid.push_back(a1);
        to_grid.push_back(a2);
        to_coeff.push_back(b1);
        to_coeff.push_back(b2);
    } else {
        const int64_t n0 = g.Ms[0], n1 = g.Ms[1];
        FftStep Rw = base(n1, n0), Cl = base(n0, n1);
        Rw.pass.in_qs = n1; Rw.pass.in_is = 1; Rw.pass.out_qs = n1; Rw.pass.out_ks = 1;
        Cl.pass.in_qs = 1; Cl.pass.in_is = n1; Cl.pass.in_rowfast = 1;
        Cl.pass.out_qs = 1; Cl.pass.out_ks = n1; Cl.pass.out_rowfast = 1;
        FftStep a1 = Rw, a2 = Cl, b1 = Rw, b2 = Cl;
        a1.pass.sign = +1; a1.ld = LD_DECONV; a1.st = ST_GRID; a1.in_buf = 0; a1.out_buf = 2;
        a1.pass.in_rs = g.P; a1.pass.out_rs = g.G;
        a2.pass.sign = +1; a2.ld = LD_GRID; a2.st = ST_GRID; a2.in_buf = 2; a2.out_buf = 1;
        a2.pass.in_rs = g.G; a2.pass.out_rs = g.G;
        b1.pass.sign = -1; b1.ld = LD_HALO; b1.st = ST_GRID; b1.in_buf = 1; b1.out_buf = 2;
        b1.pass.in_rs = g.G; b1.pass.out_rs = g.G;
        b2.pass.sign = -1; b2.ld = LD_GRID; b2.st = ST_DECONV; b2.in_buf = 2; b2.out_buf = 0;
        b2.pass.in_rs = g.G; b2.pass.out_rs = g.P;
        to_grid.push_back(a1);
        to_grid.push_back(a2);
        to_coeff.push_back(b1);
        to_coeff.push_back(b2);
    }
    // rows per workgroup found by the autotuner
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<FftStep>& v = dir == 0 ? to_grid : to_coeff;
        for (size_t k = 0; k < v.size() && k < 2; ++k) {
            const int want = P->fft_rows[dir][k];
            if (want > 0) v[k].pass.rows = std::max(1, std::min<int>(want, cap / v[k].pass.n));
        }
    }
    return INFFT_OK;
}

int run_fft(infft_plan_s* P, const std::vector<FftStep>& steps, const void* user_in, void* user_out,
            bool inv = false, void* buf1 = nullptr, void* buf2 = nullptr) {
    const Geo& g = P->g;
    for (const FftStep& s : steps) {
        FftIO io{};
        auto buf = [&](int which, bool input) -> void* {
            if (which == 0) return input ? (void*)user_in : user_out;
            if (which == 1) return buf1 ? buf1 : P->grid;
            return buf2 ? buf2 : P->grid2;
        };
        io.in = buf(s.in_buf, true);
        io.out = buf(s.out_buf, false);
        const bool f32 = P->prec == INFFT_F32;
        float* const* D32 = inv ? P->Di32 : P->D32;
        double* const* D64 = inv ? P->Di64 : P->D64;
        io.D0 = f32 ? (const void*)D32[0] : (const void*)D64[0];
        io.D1 = f32 ? (const void*)D32[1] : (const void*)D64[1];
        io.h0 = P->h0;
        io.h1 = P->h1;
        io.h01 = P->h01;
        io.halo_rs0 = P->hrs0;
        io.halo_rs1 = P->hrs1;
        io.halo_rs01 = P->hrs01;
        ProfScope ps(P, INFFT_K_FFT);
        if (f32) launch_fft_pass<float>(s.pass, io, g, s.ld, s.st, P->stream);
        else launch_fft_pass<double>(s.pass, io, g, s.ld, s.st, P->stream);
        LAUNCH_CHECK();
    }
    return INFFT_OK;
}

// Kaiser-Bessel window in grid units (host, long double): sinh(b t) / (pi t), t = sqrt(m^2 - v^2).
long double kb_window_host(long double v, int m, long double b) {
    const long double t2 = ((long double)m - v) * ((long double)m + v);
    if (t2 < 0) return 0.0L;
    const long double t = sqrtl(t2);
    const long double pi = 3.14159265358979323846264338327950288L;
    return t > 0 ? sinhl(b * t) / (pi * t) : b / pi;
}

// Monomial coefficients (ascending powers of y in [-1, 1]) of the degree nc-1 polynomial that
// interpolates w(m - 1 + (y + 1)/2 - tau) at the Chebyshev points, for taps tau = 0 .. 2m-1.
std::vector<long double> window_poly_coeffs(int m, long double b, int nc) {
    const int D = nc - 1;
    const long double pi = 3.14159265358979323846264338327950288L;
    std::vector<long double> out((size_t)2 * m * nc, 0.0L);
    for (int tau = 0; tau < 2 * m; ++tau) {
        std::vector<long double> f(nc), c(nc, 0.0L);
        for (int j = 0; j < nc; ++j) {
            const long double y = cosl(pi * (j + 0.5L) / nc);
            f[j] = kb_window_host((long double)(m - 1) + (y + 1.0L) / 2.0L - tau, m, b);
        }
        for (int k = 0; k < nc; ++k) {
            long double acc = 0.0L;
            for (int j = 0; j < nc; ++j) acc += f[j] * cosl(pi * k * (j + 0.5L) / nc);
            c[k] = acc * 2.0L / nc;
        }
        c[0] *= 0.5L;
        // sum_k c_k T_k(y) -> monomials, with T_{k+1} = 2 y T_k - T_{k-1}
        std::vector<long double> Tm(nc, 0.0L), T0(nc, 0.0L), T1(nc, 0.0L), mono(nc, 0.0L);
        T0[0] = 1.0L;
        if (D >= 1) T1[1] = 1.0L;
        for (int i = 0; i < nc; ++i) mono[i] += c[0] * T0[i];
        if (D >= 1)
            for (int i = 0; i < nc; ++i) mono[i] += c[1] * T1[i];
        for (int k = 2; k <= D; ++k) {
            std::vector<long double> T2(nc, 0.0L);
            for (int i = 0; i + 1 < nc; ++i) T2[i + 1] += 2.0L * T1[i];
            for (int i = 0; i < nc; ++i) T2[i] -= T0[i];
            for (int i = 0; i < nc; ++i) mono[i] += c[k] * T2[i];
            T0 = T1;
            T1 = T2;
        }
        (void)D;
        for (int i = 0; i < nc; ++i) out[(size_t)tau * nc + i] = mono[i];
    }
    return out;
}

int auto_tile(int Ms, int m, int want) {
    for (int t = std::min(Ms, want); t >= 2 * m; --t)
        if (Ms % t == 0) return t;
    return 0;
}

// Records what the current slot's grid holds: the oversampled F D fhat of an nfft_trafo of
// `trafo_rhs` right-hand sides, or (0) anything else.  all_slots: every slot (node changes,
// autotuning).
static void grid_holds(infft_plan_s* p, int trafo_rhs, bool all_slots = false) {
    if (!p || p->batch || p->slots.empty()) return;
    if (all_slots) {
        for (auto& sl : p->slots) sl.trafo_rhs = 0;
        return;
    }
    p->slots[p->cur_slot].trafo_rhs = trafo_rhs;
}

int set_nodes_impl(infft_plan_s* P, const double* x) {
    const Geo& g = P->g;
    hipStream_t s = P->stream;
    ProfScope ps(P, INFFT_K_NODES);
    grid_holds(P, 0, true);
    // the cell sort leaves the counters and fill cursors at zero for the next call; the plan's
    // first call (fresh allocations) zeroes them first
    if (!P->nodes_zeroed) {
        launch_nodes_reset(P->status, P->counts, g.G + 1, P->fill, g.G, P->lcount, s);
        P->nodes_zeroed = true;
    }
    launch_prep_nodes(g, x, P->nd, P->counts, P->nonfinite, s);
    launch_sort_nodes(g, P->nd, P->counts, P->fill, P->bsum, P->nonfinite, P->status, s);
    if (g.d == 2) launch_spread_worklist(g, P->nd, P->spwork, P->sp_offs, P->sp_bsum, s);
    LAUNCH_CHECK();
    P->bopt_ready = false;
    return INFFT_OK;
}

int check_rhs(infft_plan_s* P, int nrhs) {
    if (!P) return fail(INFFT_EINVAL, "null plan");
    if (nrhs < 1) return fail(INFFT_EINVAL, "nrhs must be >= 1 (got %d)", nrhs);
    return INFFT_OK;
}

// Schedules are built per chunk size (the number of sequences enters the pass descriptors).
int schedule_for(infft_plan_s* P, int rc) {
    return build_schedule(P, rc, P->to_grid, P->to_coeff);
}

// Plain DFTs of length M_sigma (1-D plans) over `nrhs` rows in grid order,
// out[r][l] = sum_s in[r][s] e^{sign 2 pi i s l / M_sigma}: the plan's own passes with grid loads and
// stores; buffer 0 in and out, buffer 2 between the two passes of a split length.
int build_plain_fft(infft_plan_s* P, int nrhs, int sign, std::vector<FftStep>& steps) {
    std::vector<FftStep> tg, tc;
    int rc = build_schedule(P, nrhs, tg, tc);
    if (rc) return rc;
    const int64_t G = P->g.G;
    steps = sign > 0 ? tg : tc;
    for (size_t i = 0; i < steps.size(); ++i) {
        FftStep& st = steps[i];
        const bool last = i + 1 == steps.size();
        st.pass.sign = sign;
        st.ld = LD_GRID;
        st.st = last ? ST_GRID : ST_TWIDDLE;
        st.in_buf = i == 0 ? 0 : 2;
        st.out_buf = last ? 0 : 2;
        st.pass.in_rs = G;
        st.pass.out_rs = G;
    }
    return INFFT_OK;
}

KTabDev plan_ktab(const infft_plan_s* p) {
    const Geo& g = p->g;
    KTabDev kt{};
    for (int t = 0; t < MAX_D; ++t) {
        kt.K[t] = p->Ktab[t];
        kt.Q[t] = p->Qtab[t];
    }
    kt.Ks = p->Kstab;
    kt.Qs = p->Qstab;
    kt.dM = p->dM;
    kt.inv_sigma = (double)g.M[0] / (double)g.Ms[0];
    kt.qK = p->qK;
    kt.qQ = p->qQ;
    kt.lam = p->lam;
    kt.scaleG = (double)g.G;
    return kt;
}

// Carves `count` elements of T from a workspace region [base + used, base + size).
template <typename T>
int carve(char* base, int64_t size, int64_t& used, T** p, int64_t count) {
    const int64_t off = (used + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
    const int64_t nb = std::max<int64_t>(count, 1) * (int64_t)sizeof(T);
    if (off + nb > size)
        return fail(INFFT_ENOMEM, "the workspace kept for large local problems (%lld bytes) is too small: "
                    "%lld bytes needed (option large_mib)", (long long)size, (long long)(off + nb));
    *p = (T*)(base + off);
    used = off + nb;
    return INFFT_OK;
}

// Records the large-problem pass for the problems the last tier listed (count and list on the
// device): reads the count and the sizes back, sorts the problems by size, packs them into
// batches whose matrices fit the workspace, and uploads problem descriptors and task lists of
// every batch.  Synchronises the stream.
int big_record(infft_plan_s* p, BigSched& S, const int* list, const int* count_dev) {
    const Geo& g = p->g;
    hipStream_t st = p->stream;
    int rc;
    S.built = false;
    S.batches.clear();
    // a new generation: graphs that replay an earlier record find it stale on the device
    S.gen += 1;
    int count = 0;
    HIP_TRY(hipMemcpyAsync(&count, count_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!S.slot && (rc = p->alloc(&S.slot, g.G))) return rc;
    if (!S.flag && (rc = p->alloc(&S.flag, 2))) return rc;
    launch_fill_i32(S.slot, g.G, -1, st);
    launch_fill_i32(S.flag + 1, 1, S.gen, st);
    LAUNCH_CHECK();
    S.count = count;
    if (count <= 0) {
        S.built = true;
        return INFFT_OK;
    }
    if (!p->big_n && (rc = p->alloc(&p->big_n, g.G))) return rc;
    launch_big_count(g, p->nd, list, count, p->big_n, st);
    LAUNCH_CHECK();
    std::vector<int> ls(count), ns(count);
    HIP_TRY(hipMemcpyAsync(ls.data(), list, sizeof(int) * count, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ns.data(), p->big_n, sizeof(int) * count, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return ns[a] != ns[b] ? ns[a] > ns[b] : ls[a] < ls[b];
    });
    S.nmax = ns[order.front()];
    S.nmin = ns[order.back()];
    // batch budget for matrices and member data (40 bytes per member).  Ordinary plans: a quarter
    // of the free device memory, between 1 and 16 GiB (every batch runs its block steps in sequence,
    // so fewer, larger batches shorten the chain of dependent launches); workspace plans: three
    // quarters of the part of the workspace kept for large problems, the rest for the descriptors
    // and task lists of both records.
    int64_t budget;
    if (p->ws_mode) {
        budget = p->large_arena_bytes / 4 * 3;
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
        budget = std::min<int64_t>(std::max<int64_t>((int64_t)(free_b / 4), (int64_t)1 << 30), (int64_t)16 << 30);
    }
    const int64_t one = (int64_t)S.nmax * S.nmax * 16 + (int64_t)S.nmax * 40 + 4096;
    if (p->ws_mode && one > budget)
        return fail(INFFT_ENOMEM, "a local problem of %d members needs %lld bytes; the workspace keeps %lld for "
                    "large problems (option large_mib)", S.nmax, (long long)one, (long long)budget);
    const int64_t cap_bytes = std::max<int64_t>(budget, one);
    std::vector<BigProb> probs;
    std::vector<int4> tasks;
    probs.reserve(count);
    int64_t maxA = 1, maxM = 1;
    size_t pos = 0;
    while (pos < order.size()) {
        BigBatch b;
        b.prob_off = (int64_t)probs.size();
        int64_t ent = 0, mem = 0;
        while (pos < order.size()) {
            const int q = order[pos];
            const int64_t n = ns[q];
            const int64_t e = (n * n + 31) / 32 * 32;
            if (b.np > 0 && (ent + e) * 16 + (mem + n) * 40 > cap_bytes) break;
            BigProb bp{};
            bp.l = ls[q];
            bp.n = (int)n;
            bp.nblk = (int)((n + BIG_NB - 1) / BIG_NB);
            bp.id = (int)probs.size();   // index of the failure flag: position in the sorted order
            bp.off = ent;
            bp.moff = mem;
            probs.push_back(bp);
            b.nblk.push_back(bp.nblk);
            ent += e;
            mem += n;
            ++b.np;
            ++pos;
        }
        maxA = std::max(maxA, ent);
        maxM = std::max(maxM, mem);
        b.T0 = b.nblk.front();
        const BigProb* pb = probs.data() + b.prob_off;
        // task lists: Gram tiles, then per block column k the panel and trailing tiles
        b.seg.push_back((int64_t)tasks.size());
        for (int i = 0; i < b.np; ++i)
            for (int I = 0; I < pb[i].nblk; ++I)
                for (int J = 0; J <= I; ++J) tasks.push_back(make_int4(i, I, J, 0));
        for (int k = 0; k < b.T0; ++k) {
            b.seg.push_back((int64_t)tasks.size());
            for (int i = 0; i < b.np && pb[i].nblk > k; ++i)
                for (int I = k + 1; I < pb[i].nblk; ++I) tasks.push_back(make_int4(i, I, 0, 0));
            b.seg.push_back((int64_t)tasks.size());
            for (int i = 0; i < b.np && pb[i].nblk > k; ++i)
                for (int I = k + 1; I < pb[i].nblk; ++I)
                    for (int J = k + 1; J <= I; ++J) tasks.push_back(make_int4(i, I, J, 0));
        }
        b.seg.push_back((int64_t)tasks.size());
        // substitution steps (right-looking, one launch per block step): forward (problem, I >= k),
        // backward (problem, J <= k)
        for (int k = 0; k < b.T0; ++k) {
            b.fseg.push_back((int64_t)tasks.size());
            for (int i = 0; i < b.np && pb[i].nblk > k; ++i)
                for (int I = k; I < pb[i].nblk; ++I) tasks.push_back(make_int4(i, I, 0, 0));
        }
        b.fseg.push_back((int64_t)tasks.size());
        for (int k = 0; k < b.T0; ++k) {
            b.bseg.push_back((int64_t)tasks.size());
            for (int i = 0; i < b.np && pb[i].nblk > k; ++i)
                for (int J = 0; J <= k; ++J) tasks.push_back(make_int4(i, J, 0, 0));
        }
        b.bseg.push_back((int64_t)tasks.size());
        S.batches.push_back(std::move(b));
    }
    const int64_t ntask = std::max<int64_t>((int64_t)tasks.size(), 1);
    // device arrays: the shared matrices and member data, this record's descriptors and tasks
    if (p->ws_mode) {
        char* base = p->large_arena;
        int64_t used = 0;
        const int64_t wsz = budget;
        if ((rc = carve(base, wsz, used, &p->big_A, maxA)) || (rc = carve(base, wsz, used, &p->big_midx, maxM)) ||
            (rc = carve(base, wsz, used, &p->big_mtap, maxM)) || (rc = carve(base, wsz, used, &p->big_mz, maxM)) ||
            (rc = carve(base, wsz, used, &p->big_mr, maxM)) || (rc = carve(base, wsz, used, &p->big_mb, maxM)))
            return rc;
        // each record owns one eighth of the part kept for large problems
        const int64_t rsz = p->large_arena_bytes / 8;
        char* rbase = base + budget + (int64_t)(&S - p->big_sched) * rsz;
        int64_t rused = 0;
        if ((rc = carve(rbase, rsz, rused, &S.probs, count)) || (rc = carve(rbase, rsz, rused, &S.tasks, ntask)) ||
            (rc = carve(rbase, rsz, rused, &S.fail, count)))
            return rc;
    } else {
        if ((rc = p->grow_retire(&p->big_A, p->big_A_cap, maxA))) return rc;
        if (maxM > p->big_m_cap) {
            int64_t c1 = p->big_m_cap, c2 = p->big_m_cap, c3 = p->big_m_cap, c4 = p->big_m_cap,
                    c5 = p->big_m_cap;
            if ((rc = p->grow_retire(&p->big_midx, c1, maxM)) || (rc = p->grow_retire(&p->big_mtap, c2, maxM)) ||
                (rc = p->grow_retire(&p->big_mz, c3, maxM)) || (rc = p->grow_retire(&p->big_mr, c4, maxM)) ||
                (rc = p->grow_retire(&p->big_mb, c5, maxM)))
                return rc;
            p->big_m_cap = c1;
        }
        if ((rc = p->grow_retire(&S.probs, S.probs_cap, count)) ||
            (rc = p->grow_retire(&S.tasks, S.tasks_cap, ntask)) || (rc = p->grow_retire(&S.fail, S.fail_cap, count)))
            return rc;
    }
    HIP_TRY(hipMemcpy(S.probs, probs.data(), sizeof(BigProb) * probs.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(S.tasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice));
    launch_big_slots(S.probs, count, S.slot, st);
    LAUNCH_CHECK();
    S.built = true;
    return INFFT_OK;
}

// Enqueues a recorded large-problem pass (no host synchronisation: also under graph capture).
// A check kernel first compares the problems the last tier listed with the record; if they differ
// (the nodes changed since the record), every large-problem kernel returns at once and the listed
// problems get zero columns and are counted as oversized.  grad: the node-gradient pass instead of
// the solutions.  Adds one statistics record for the precompute.
int big_enqueue(infft_plan_s* p, BigSched& S, const KTabDev& kt, const int* list, const int* count_dev,
                int& stat_off, const BoptGradArgs* grad, bool capturing) {
    const Geo& g = p->g;
    hipStream_t st = p->stream;
    if (S.count == 0) {
        // nothing recorded: outside capture the count was just read back, so there is nothing to
        // do; under capture one kernel checks that the tiers still list no problem (and that the
        // record is current), else zeroes the listed problems' columns and counts them
        if (capturing && !grad) {
            launch_big_guard_empty(g, p->nd, list, count_dev, S.flag + 1, S.gen, p->out_B64, p->out_B32, p->stat_rec,
                                   p->status, st);
            LAUNCH_CHECK();
        }
        return INFFT_OK;
    }
    // outside capture the record was just made from these lists: no check
    if (capturing) {
        launch_fill_i32(S.flag, 1, 0, st);
        launch_big_check(g, p->nd, list, count_dev, S.slot, S.probs, S.count, S.gen, S.flag, st);
        LAUNCH_CHECK();
    }
    {
        launch_fill_i32(S.fail, S.count, 0, st);
        BigArgs a{};
        a.A = p->big_A;
        a.midx = p->big_midx;
        a.mtap = p->big_mtap;
        a.mz = p->big_mz;
        a.mr = p->big_mr;
        a.mb = p->big_mb;
        a.fail = S.fail;
        a.stale = capturing ? S.flag : nullptr;
        for (const BigBatch& b : S.batches) {
            a.probs = S.probs + b.prob_off;
            launch_big_setup(g, p->nd, kt, a, b.np, st);
            LAUNCH_CHECK();
            launch_big_gram(g, kt, a, S.tasks + b.seg[0], (int)(b.seg[1] - b.seg[0]), st);
            LAUNCH_CHECK();
            int active = b.np;
            for (int k = 0; k < b.T0; ++k) {
                while (active > 0 && b.nblk[active - 1] <= k) --active;
                launch_big_potrf(a, active, k, st);
                LAUNCH_CHECK();
                const int64_t t0 = b.seg[1 + 2 * k], t1 = b.seg[2 + 2 * k], t2 = b.seg[3 + 2 * k];
                launch_big_trsm(a, S.tasks + t0, (int)(t1 - t0), k, st);
                LAUNCH_CHECK();
                launch_big_herk(a, S.tasks + t1, (int)(t2 - t1), k, st);
                LAUNCH_CHECK();
            }
            if (grad) {
                launch_big_grad(g, a, kt, *grad, p->nd.perm, b.np, p->prec == INFFT_F32, st);
            } else {
                for (int k = 0; k < b.T0; ++k) {
                    launch_big_fwd(a, S.tasks + b.fseg[k], (int)(b.fseg[k + 1] - b.fseg[k]), k, st);
                    LAUNCH_CHECK();
                }
                for (int k = b.T0 - 1; k >= 0; --k) {
                    launch_big_bwd(a, S.tasks + b.bseg[k], (int)(b.bseg[k + 1] - b.bseg[k]), k, st);
                    LAUNCH_CHECK();
                }
                launch_big_write(g, a, b.np, p->out_B64, p->out_B32, st);
            }
            LAUNCH_CHECK();
        }
    }
    if (grad) return INFFT_OK;   // the precompute's statistics stay as they are
    if (capturing) {
        launch_big_zero_stale(g, p->nd, list, count_dev, S.flag, p->out_B64, p->out_B32, p->stat_rec, p->status, st);
        LAUNCH_CHECK();
    }
    launch_big_stats(S.fail, S.count, S.nmin, S.nmax, p->stat_rec + (int64_t)stat_off * 5, st);
    LAUNCH_CHECK();
    stat_off += 1;
    return INFFT_OK;
}

// Local problems with more members than the register tiers hold (list of grid indices and its
// device count from the last tier): recorded anew outside graph capture, replayed from the last
// record under capture or when `replay` asks for it (INFFT_ESTATE when there is none).  Record 0
// serves the precompute, record 1 the node gradient through B_opt(x), whose tiers pass on a
// different set of problems.
int solve_large(infft_plan_s* p, const KTabDev& kt, const int* list, const int* count_dev, int& stat_off,
                const BoptGradArgs* grad = nullptr, bool replay = false) {
    BigSched& S = p->big_sched[grad ? 1 : 0];
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(p->stream, &cs));
    const bool capturing = replay || cs != hipStreamCaptureStatusNone;
    if (!capturing) {
        int rc = big_record(p, S, list, count_dev);
        if (rc) return rc;
    } else if (!S.built) {
        return fail(INFFT_ESTATE, "under graph capture the pass for local problems beyond the register tiers "
                    "replays the one recorded by the last call outside capture, and there is none yet");
    }
    return big_enqueue(p, S, kt, list, count_dev, stat_off, grad, capturing);
}

}  // namespace

// ------------------------------------------------------------------ many 1-D problems in one plan
// A batch plan owns one ordinary plan per problem (its nodes, grid, tables, B_opt, lists) and
// launch tables that let every stage run for all problems in one launch: per launch an array of
// per-problem arguments ("jobs") and a map workgroup -> (job, block of that job).  Caller arrays
// are problem-major: coefficients [problem][nrhs][M_i], samples [problem][nrhs][N_i].

struct BatchLaunch {
    int ld = 0, st = 0;
    bool small = false;   // FP32 passes in the small-capacity kernel
    int64_t map_off = 0;
    int nblocks = 0;
    size_t shm = 0;
};

struct BatchState {
    std::vector<infft_plan_s*> subs;
    std::vector<int64_t> Poff, Noff;
    int64_t Ptot = 0, Ntot = 0;
    FftJob* fft_jobs = nullptr;
    FftJob* fft_jobs_inv = nullptr;   // the same passes with the inverse's factors
    int2* fft_map = nullptr;
    std::vector<BatchLaunch> to_grid, to_coeff;
    NodeJob* node_jobs = nullptr;
    int2* node_map = nullptr;
    int node_blocks = 0;
    int2* cell_map = nullptr;   // tiles of the 1-D spreading
    int cell_blocks = 0;
    SolveJob* solve_jobs = nullptr;   // [5][nprob]: thread tier, 16, 32 and 64 lanes, 64 lanes under capture
    int2* t1_map = nullptr;
    int t1_blocks = 0;
    std::vector<int> t1_per_prob;
    int tier_blocks = 1024;
    int* counts = nullptr;
};

void batch_free(BatchState* b) {
    for (infft_plan_s* s : b->subs) {
        if (s) {
            (void)hipStreamSynchronize(s->stream);
            delete s;
        }
    }
    delete b;
}

namespace {

template <typename T>
int upload(infft_plan_s* P, T** dst, const std::vector<T>& v) {
    int rc = P->alloc(dst, (int64_t)std::max<size_t>(v.size(), 1));
    if (rc) return rc;
    if (!v.empty()) HIP_TRY(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return INFFT_OK;
}

// Launch tables of the batch plan P from its per-problem plans.
int batch_build(infft_plan_s* P) {
    BatchState& B = *P->batch;
    const int np = (int)B.subs.size();
    const size_t cs = P->csize();
    // ---- FFT passes, grouped by (step index, load mode, store mode, kernel).  FP32 passes of
    // sub-transforms up to the small kernel's capacity go to that kernel, with at most that many
    // elements per workgroup (the rows do not change the arithmetic).
    std::vector<FftJob> jobs, jobs_inv;
    std::vector<int2> map;
    const int small_cap = fft_batched_small_capacity();
    for (int dir = 0; dir < 2; ++dir) {
        std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
        for (int i = 0; i < np; ++i) {
            infft_plan_s* sub = B.subs[i];
            std::vector<FftStep> tg, tc;
            sub->fft_min_blocks = 1;
            int rc = build_schedule(sub, sub->max_rhs, tg, tc);
            sub->fft_min_blocks = 1024;
            if (rc) return rc;
            const std::vector<FftStep>& steps = dir == 0 ? tg : tc;
            for (size_t k = 0; k < steps.size(); ++k) {
                const FftStep& st = steps[k];
                FftJob J{};
                J.pass = st.pass;
                J.g = sub->g;
                const bool f32 = sub->prec == INFFT_F32;
                J.io.in = st.in_buf == 1 ? sub->grid : st.in_buf == 2 ? sub->grid2 : nullptr;
                J.io.out = st.out_buf == 1 ? sub->grid : st.out_buf == 2 ? sub->grid2 : nullptr;
                J.io.D0 = f32 ? (const void*)sub->D32[0] : (const void*)sub->D64[0];
                J.io.D1 = nullptr;
                J.user_in = st.in_buf == 0;
                J.user_out = st.out_buf == 0;
                J.user_off = B.Poff[i];
                const bool small = f32 && J.pass.n <= small_cap;
                if (small) J.pass.rows = std::max(1, std::min(J.pass.rows, small_cap / J.pass.n));
                groups[std::make_tuple((int)k, st.ld, st.st, (int)small)].push_back((int)jobs.size());
                jobs.push_back(J);
                J.io.D0 = f32 ? (const void*)sub->Di32[0] : (const void*)sub->Di64[0];
                jobs_inv.push_back(J);
            }
        }
        std::vector<BatchLaunch>& launches = dir == 0 ? B.to_grid : B.to_coeff;
        launches.clear();
        for (auto& kv : groups) {
            BatchLaunch L;
            L.ld = std::get<1>(kv.first);
            L.st = std::get<2>(kv.first);
            L.small = std::get<3>(kv.first) != 0;
            L.map_off = (int64_t)map.size();
            for (int ji : kv.second) {
                const FftPass& ps = jobs[ji].pass;
                const int64_t nb = (ps.nseq + ps.rows - 1) / ps.rows;
                for (int64_t b = 0; b < nb; ++b) map.push_back(make_int2(ji, (int)b));
                L.shm = std::max(L.shm, fft_lds_bytes(ps, cs));
            }
            L.nblocks = (int)((int64_t)map.size() - L.map_off);
            launches.push_back(L);
        }
    }
    int rc;
    if ((rc = upload(P, &B.fft_jobs, jobs)) || (rc = upload(P, &B.fft_map, map))) return rc;
    if (B.subs[0]->inv_kernel == INFFT_KERNEL_WINDOW) B.fft_jobs_inv = B.fft_jobs;
    else if ((rc = upload(P, &B.fft_jobs_inv, jobs_inv))) return rc;
    // ---- per-node and per-cell kernels
    std::vector<NodeJob> nj(np);
    std::vector<int2> nmap, cmap, tmap;
    B.t1_per_prob.assign(np, 0);
    for (int i = 0; i < np; ++i) {
        infft_plan_s* sub = B.subs[i];
        NodeJob& J = nj[i];
        J.g = sub->g;
        J.nd = sub->nd;
        J.B = sub->prec == INFFT_F32 ? (const void*)sub->B32 : (const void*)sub->B64;
        J.grid = sub->grid;
        J.grs = sub->g.G;
        J.noff = B.Noff[i];
        for (int64_t b = 0; b < (sub->g.N + 255) / 256; ++b) nmap.push_back(make_int2(i, (int)b));
        for (int b = 0; b < spread1d_tiles(sub->g); ++b) cmap.push_back(make_int2(i, b));
        const int nt = (int)((sub->g.G + T1_CELLS - 1) / T1_CELLS);
        B.t1_per_prob[i] = nt;
        for (int b = 0; b < nt; ++b) tmap.push_back(make_int2(i, b));
    }
    B.node_blocks = (int)nmap.size();
    B.cell_blocks = (int)cmap.size();
    B.t1_blocks = (int)tmap.size();
    if ((rc = upload(P, &B.node_jobs, nj)) || (rc = upload(P, &B.node_map, nmap)) ||
        (rc = upload(P, &B.cell_map, cmap)) || (rc = upload(P, &B.t1_map, tmap)))
        return rc;
    // ---- solver tiers: thread per problem, then the 16-, 32- and 64-member tiers over each
    // problem's lists
    std::vector<SolveJob> sj(5 * (size_t)np);
    for (int i = 0; i < np; ++i) {
        infft_plan_s* sub = B.subs[i];
        SolveJob base{};
        base.g = sub->g;
        base.nd = sub->nd;
        base.kt = plan_ktab(sub);
        // a batch keeps both copies of B_opt (its get_B reads the FP64 one directly)
        sub->out_B64 = base.a.B64 = sub->B64;
        sub->out_B32 = base.a.B32 = sub->B32;
        base.a.status = sub->status;
        base.a.stat_rec = sub->stat_rec;
        int* listA = sub->lists;
        int* listB = sub->lists + sub->g.G;
        SolveJob t0 = base, t1 = base, t2 = base, t3 = base;
        t0.a.out_list = listA;
        t0.a.out_count = sub->lcount;
        t0.a.out_list2 = listB;   // 17 to 32 members: straight to the 32-member tier's list
        t0.a.out_count2 = sub->lcount + 1;
        t0.a.stat_off = 0;
        t1.a.in_list = listA;
        t1.a.in_count = sub->lcount;
        t1.a.out_list = listB;
        t1.a.out_count = sub->lcount + 1;
        t1.a.stat_off = B.t1_per_prob[i];
        t2.a.in_list = listB;
        t2.a.in_count = sub->lcount + 1;
        t2.a.out_list = listA;
        t2.a.out_count = sub->lcount + 2;
        t2.a.stat_off = B.t1_per_prob[i] + 1;
        t3.a.in_list = listA;
        t3.a.in_count = sub->lcount + 2;
        t3.a.out_list = listB;
        t3.a.out_count = sub->lcount + 3;
        t3.a.stat_off = B.t1_per_prob[i] + 2;
        SolveJob t4 = t3;
        t4.a.out_list = nullptr;
        t4.a.out_count = nullptr;
        sj[i] = t0;
        sj[np + i] = t1;
        sj[2 * (size_t)np + i] = t2;
        sj[3 * (size_t)np + i] = t3;
        sj[4 * (size_t)np + i] = t4;
    }
    if ((rc = upload(P, &B.solve_jobs, sj))) return rc;
    if ((rc = P->alloc(&B.counts, np))) return rc;
    return INFFT_OK;
}

int run_fft_batched(infft_plan_s* P, const std::vector<BatchLaunch>& launches, const void* user_in,
                    void* user_out, int nrhs, bool inv = false) {
    BatchState& B = *P->batch;
    const FftJob* jobs = inv ? B.fft_jobs_inv : B.fft_jobs;
    for (const BatchLaunch& L : launches) {
        ProfScope ps(P, INFFT_K_FFT);
        if (P->prec == INFFT_F32)
            launch_fft_batched<float>(jobs, B.fft_map + L.map_off, L.nblocks, L.shm, L.ld, L.st, user_in,
                                      user_out, nrhs, L.small, P->stream);
        else
            launch_fft_batched<double>(jobs, B.fft_map + L.map_off, L.nblocks, L.shm, L.ld, L.st, user_in,
                                       user_out, nrhs, false, P->stream);
        LAUNCH_CHECK();
    }
    return INFFT_OK;
}

int node_batched(infft_plan_s* P, int kind, const void* in, void* out, double* gradx, int nrhs) {
    BatchState& B = *P->batch;
    const bool cells = kind == NB_GATHER || kind == NB_GATHER_B;
    const int2* map = cells ? B.cell_map : B.node_map;
    const int nb = cells ? B.cell_blocks : B.node_blocks;
    ProfScope ps(P, cells ? INFFT_K_SPREAD : INFFT_K_INTERP);
    if (P->prec == INFFT_F32)
        launch_node_batched<float>(kind, P->g.m, B.node_jobs, map, nb, (const float2*)in, (float2*)out, gradx, nrhs,
                                   0, P->stream);
    else
        launch_node_batched<double>(kind, P->g.m, B.node_jobs, map, nb, (const double2*)in, (double2*)out, gradx,
                                    nrhs, 0, P->stream);
    LAUNCH_CHECK();
    return INFFT_OK;
}

int batch_check_rhs(infft_plan_s* P, int nrhs) {
    if (nrhs < 1) return fail(INFFT_EINVAL, "nrhs must be positive");
    if (nrhs > P->max_rhs) return fail(INFFT_ESTATE, "a batch plan takes at most max_rhs = %d right-hand sides", P->max_rhs);
    return INFFT_OK;
}

int batch_precompute(infft_plan_s* P) {
    BatchState& B = *P->batch;
    const int np = (int)B.subs.size();
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(P->stream, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    P->bopt_ready = false;
    launch_batch_solve_reset(B.solve_jobs, np, P->stream);
    LAUNCH_CHECK();
    {
        ProfScope ps(P, INFFT_K_SOLVE);
        launch_solve_t1_batched(B.solve_jobs, B.t1_map, B.t1_blocks, B.subs[0]->qQ, B.subs[0]->qK, P->stream);
    }
    LAUNCH_CHECK();
    launch_solve_tier_batched(B.solve_jobs + np, np, 16, B.tier_blocks, P->stream);
    LAUNCH_CHECK();
    launch_solve_tier_batched(B.solve_jobs + 2 * (size_t)np, np, 32, B.tier_blocks, P->stream);
    LAUNCH_CHECK();
    launch_solve_tier_batched(B.solve_jobs + (capturing ? 4 : 3) * (size_t)np, np, 64, B.tier_blocks, P->stream);
    LAUNCH_CHECK();
    for (int i = 0; i < np; ++i) {
        B.subs[i]->stat_nrec = B.t1_per_prob[i] + 3;   // three list tiers: one record each
        B.subs[i]->bopt_ready = true;
    }
    if (!capturing) {
        launch_batch_counts(B.solve_jobs + 3 * (size_t)np, np, B.counts, P->stream);
        LAUNCH_CHECK();
        std::vector<int> cnt(np);
        HIP_TRY(hipMemcpyAsync(cnt.data(), B.counts, sizeof(int) * np, hipMemcpyDeviceToHost, P->stream));
        HIP_TRY(hipStreamSynchronize(P->stream));
        for (int i = 0; i < np; ++i) {
            if (cnt[i] == 0) continue;
            infft_plan_s* sub = B.subs[i];
            int off = sub->stat_nrec;
            int rc = solve_large(sub, plan_ktab(sub), sub->lists + sub->g.G, sub->lcount + 3, off);
            if (rc) return rc;
            sub->stat_nrec = off;
        }
    }
    P->bopt_kind = 0;
    P->bopt_ready = true;
    return INFFT_OK;
}

}  // namespace


// =====================================================================================  C ABI

extern "C" {

void infft_default_options(infft_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = INFFT_F64;
    o->max_rhs = 1;
    o->rho = 1e-8;
}

const char* infft_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// A validated parameter set: geometry, options, work slots and the split of a long 1-D FFT.
struct PlanSpec {
    Geo g{};
    infft_options o{};
    double sigma = 2.0;
    int nslots = 1;
    int64_t n1_split = 0;
};

int plan_validate(int d, const int64_t* M, int64_t N, double sigma, int m, const infft_options* opts,
                  PlanSpec& S) {
    if (d < 1 || d > 2) return fail(INFFT_EINVAL, "d must be 1 or 2 (got %d)", d);
    if (!M) return fail(INFFT_EINVAL, "M is null");
    if (N <= 0 || N >= (int64_t)1 << 31) return fail(INFFT_EINVAL, "N out of range (%lld)", (long long)N);
    if (m < MIN_M_CUT || m > MAX_M_CUT) return fail(INFFT_EINVAL, "m must be in %d..%d (got %d)", MIN_M_CUT, MAX_M_CUT, m);
    if (!(sigma >= 1.0) || !std::isfinite(sigma)) return fail(INFFT_EINVAL, "sigma must be >= 1");
    infft_options& o = S.o;
    infft_default_options(&o);
    if (opts) o = *opts;
    if (o.precision != INFFT_F32 && o.precision != INFFT_F64) return fail(INFFT_EINVAL, "bad precision");
    if (o.inverse_kernel != INFFT_KERNEL_WINDOW && o.inverse_kernel != INFFT_KERNEL_DIRICHLET)
        return fail(INFFT_EINVAL, "bad inverse_kernel");
    if (o.max_rhs < 1 || o.max_rhs > 64) return fail(INFFT_EINVAL, "max_rhs must be in 1..64");
    S.nslots = o.work_slots == 0 ? 1 : o.work_slots;
    if (S.nslots < 1 || S.nslots > 8) return fail(INFFT_EINVAL, "work_slots must be in 1..8 (got %d)", o.work_slots);
    if (!(o.rho >= 0.0) || !std::isfinite(o.rho)) return fail(INFFT_EINVAL, "rho must be finite and >= 0");
    if (o.large_mib < 0 || o.large_mib > (1 << 20)) return fail(INFFT_EINVAL, "large_mib out of range");
    if (o.ansatz1 != 0 && o.ansatz1 != 1) return fail(INFFT_EINVAL, "ansatz1 must be 0 or 1");
    S.sigma = sigma;
    Geo& g = S.g;
    g.d = d;
    g.m = m;
    g.N = N;
    g.b = M_PI * (2.0 - 1.0 / sigma);
    g.G = 1;
    g.P = 1;
    for (int t = 0; t < MAX_D; ++t) {
        g.M[t] = g.Ms[t] = g.TS[t] = g.ntile[t] = 1;
    }
    for (int t = 0; t < d; ++t) {
        if (M[t] <= 0 || M[t] % 2 || M[t] > (1 << 24))
            return fail(INFFT_EINVAL, "M[%d] must be a positive even integer (got %lld)", t, (long long)M[t]);
        const double msd = sigma * (double)M[t];
        const int64_t ms = (int64_t)std::llround(msd);
        if (std::fabs(msd - (double)ms) > 1e-9 * msd || ms % 2)
            return fail(INFFT_EINVAL, "sigma*M[%d] = %g must be an even integer", t, msd);
        if (2 * m + 2 > ms) return fail(INFFT_EINVAL, "2m+2 = %d exceeds M_sigma = %lld", 2 * m + 2, (long long)ms);
        g.M[t] = (int)M[t];
        g.Ms[t] = (int)ms;
        g.G *= ms;
        g.P *= M[t];
    }
    if (g.G > ((int64_t)1 << 22)) return fail(INFFT_EINVAL, "oversampled grid too large (%lld points)", (long long)g.G);
    if (o.ansatz1 && d != 1) return fail(INFFT_EINVAL, "ansatz1 work arrays are for d = 1 plans");
    // tiles
    for (int t = 0; t < d; ++t) {
        const int want = o.tile[t] > 0 ? o.tile[t] : (d == 1 ? 256 : 32);
        const int ts = auto_tile(g.Ms[t], m, want);
        if (ts == 0 || g.Ms[t] % ts) return fail(INFFT_EINVAL, "no spreading tile >= 2m divides M_sigma[%d]", t);
        g.TS[t] = ts;
        g.ntile[t] = g.Ms[t] / ts;
    }
    // FFT feasibility
    const int cap = fft_capacity(o.precision == INFFT_F64);
    for (int t = 0; t < d; ++t) {
        std::vector<int> rad;
        if (!factor_radices(g.Ms[t], rad))
            return fail(INFFT_EINVAL, "M_sigma[%d] = %d is not a product of 2, 3, 5, 7", t, g.Ms[t]);
        if (g.Ms[t] > cap) {
            if (d == 2) return fail(INFFT_EINVAL, "2-D grids need M_sigma <= %d per dimension", cap);
            // split n = n1 n2 with both factors <= cap, as balanced as possible
            int64_t best = 0;
            for (int64_t a = 2; a <= cap; ++a) {
                if (g.Ms[t] % a) continue;
                const int64_t b = g.Ms[t] / a;
                if (b > cap) continue;
                std::vector<int> ra, rb;
                if (!factor_radices((int)a, ra) || !factor_radices((int)b, rb)) continue;
                if (!best || std::llabs(a - b) < std::llabs(best - g.Ms[t] / best)) best = a;
            }
            if (!best) return fail(INFFT_EINVAL, "M_sigma = %d cannot be split into two FFT passes", g.Ms[t]);
            S.n1_split = best;
        }
    }
    return INFFT_OK;
}

// Parameters of the two inner plans of Algorithm 3.10 (made on the first infft_precompute_Bstar):
// the Toeplitz symbol at bandwidth 2M, sigma 2, the largest cut-off; and for FP32 plans an FP64
// twin with one node for the length-M_sigma FFTs.
struct InnerSpec {
    int64_t M;
    int64_t N;
    double sigma;
    int m;
    infft_options o;
};

InnerSpec a1_symbol_spec(const Geo& g) {
    InnerSpec s{};
    infft_default_options(&s.o);
    s.o.precision = INFFT_F64;
    s.M = 2 * (int64_t)g.M[0];
    s.N = g.N;
    s.sigma = 2.0;
    s.m = std::min<int>(MAX_M_CUT, (int)(2 * s.M - 2) / 2);
    return s;
}

InnerSpec a1_twin_spec(const Geo& g, double sigma, int inv_kernel) {
    InnerSpec s{};
    infft_default_options(&s.o);
    s.o.precision = INFFT_F64;
    s.o.inverse_kernel = inv_kernel;
    s.M = g.M[0];
    s.N = 1;
    s.sigma = sigma;
    s.m = g.m;
    return s;
}

// complex128 elements of the work arrays of Algorithm 3.10
int64_t a1_work_elems(const Geo& g) {
    const int M = g.M[0], Ms = g.Ms[0];
    const int npair = Ms >= 2 * M - 1 ? 1 : 4;
    const int64_t rows = 2 * g.m + 1;
    return (rows * (3 + 2 * npair)) * Ms + 4 * (int64_t)M + g.N;
}

int plan_measure(const PlanSpec& S, size_t* bytes);

// Places every device buffer of the plan (through P->alloc: device allocations, carving from a
// caller's workspace, or only counting bytes) and fixes the host-side layout; no device work.
int plan_layout(infft_plan_s* P, const PlanSpec& S) {
    const Geo& g = S.g;
    const int d = g.d, m = g.m;
    const int64_t N = g.N;
    const int64_t Nd = N * d;
    const int T = P->taps();
    int rc;
#define LTRY(e)                 \
    do {                        \
        if ((rc = (e)) != 0) return rc; \
    } while (0)
    double* xw = nullptr;
    LTRY(P->alloc(&xw, Nd));
    P->nd.xw = xw;
    LTRY(P->alloc(&P->nd.l0c, Nd));
    LTRY(P->alloc(&P->nd.uc, Nd));
    LTRY(P->alloc(&P->nd.key, N));
    LTRY(P->alloc(&P->nd.perm, N));
    LTRY(P->alloc(&P->nd.l0s, Nd));
    LTRY(P->alloc(&P->nd.us, Nd));
    LTRY(P->alloc(&P->nd.start, g.G + 1));
    LTRY(P->alloc(&P->counts, g.G + 1));
    LTRY(P->alloc(&P->nonfinite, prep_blocks(g)));
    LTRY(P->alloc(&P->fill, g.G));
    LTRY(P->alloc(&P->bsum, scan_blocksum_len(g.G) + 1));
    LTRY(P->alloc(&P->status, STATUS_WORDS));
    // deconvolution factors and kernel tables
    P->qK = m * TAY_S + 1;
    P->qQ = 2 * m * TAY_S + 1;
    for (int t = 0; t < d; ++t) {
        LTRY(P->alloc(&P->D64[t], g.M[t]));
        if (P->prec == INFFT_F32) LTRY(P->alloc(&P->D32[t], g.M[t]));
        LTRY(P->alloc(&P->Ktab[t], (int64_t)(P->qK + 1) * TAY_NC));
        LTRY(P->alloc(&P->Qtab[t], (int64_t)(P->qQ + 1) * TAY_NC));
        if (P->inv_kernel == INFFT_KERNEL_DIRICHLET) {
            LTRY(P->alloc(&P->Di64[t], g.M[t]));
            if (P->prec == INFFT_F32) LTRY(P->alloc(&P->Di32[t], g.M[t]));
        } else {
            P->Di64[t] = P->D64[t];
            P->Di32[t] = P->D32[t];
        }
    }
    if (d == 1) {
        LTRY(P->alloc(&P->Kstab, (int64_t)(P->qK + 1) * TAY_NC));
        LTRY(P->alloc(&P->Qstab, (int64_t)(P->qQ + 1) * TAY_NC));
    }
    // FFT twiddles (filled by plan_setup)
    const int cap = fft_capacity(P->prec == INFFT_F64);
    for (int t = 0; t < d; ++t) {
        if (g.Ms[t] <= cap) {
            LTRY(reserve_tw(P, g.Ms[t]));
        } else {
            LTRY(reserve_tw(P, S.n1_split));
            LTRY(reserve_tw(P, g.Ms[t] / S.n1_split));
            int64_t Bsz = 1;   // power of two near sqrt(M_sigma): the split of a twiddle exponent is a shift
            while (Bsz * Bsz < g.Ms[t]) Bsz *= 2;
            P->split_lo.n = Bsz;
            P->split_hi.n = S.n1_split;  // remembered sub-length of the first pass
            const int64_t nhi = (g.Ms[t] + Bsz - 1) / Bsz;
            LTRY(P->alloc(&P->split_lo.t64, Bsz));
            LTRY(P->alloc(&P->split_hi.t64, nhi));
            if (P->prec == INFFT_F32) {
                LTRY(P->alloc(&P->split_lo.t32, Bsz));
                LTRY(P->alloc(&P->split_hi.t32, nhi));
            }
        }
    }
    // window polynomials (coefficients fitted here, uploaded by plan_setup)
    {
        const int nc = P->prec == INFFT_F32 ? WPoly<float>::NC : WPoly<double>::NC;
        P->wpoly_host = window_poly_coeffs(m, (long double)M_PI * (2.0L - 1.0L / S.sigma), nc);
        if (P->prec == INFFT_F32) {
            float* dptr = nullptr;
            LTRY(P->alloc(&dptr, (int64_t)P->wpoly_host.size()));
            P->g.wpoly = dptr;
        } else {
            double* dptr = nullptr;
            LTRY(P->alloc(&dptr, (int64_t)P->wpoly_host.size()));
            P->g.wpoly = dptr;
        }
    }
    // grids, halos, B_opt, solver lists
    const size_t cs = P->csize();
    const int64_t ntiles = (int64_t)g.ntile[0] * g.ntile[1];
    const int w2 = 2 * m;
    P->hrs0 = ntiles * w2 * (d == 2 ? g.TS[1] : 1);
    P->hrs1 = d == 2 ? ntiles * g.TS[0] * w2 : 0;
    P->hrs01 = d == 2 ? ntiles * w2 * w2 : 0;
    for (int k = 0; k < S.nslots; ++k) {
        char* tmp = nullptr;
        infft_plan_s::Slot sl{};
        LTRY(P->alloc(&tmp, (int64_t)cs * g.G * P->max_rhs));
        sl.grid = tmp;
        LTRY(P->alloc(&tmp, (int64_t)cs * g.G * P->max_rhs));
        sl.grid2 = tmp;
        LTRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(P->hrs0, 1) * P->max_rhs));
        sl.h0 = tmp;
        LTRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(P->hrs1, 1) * P->max_rhs));
        sl.h1 = tmp;
        LTRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(P->hrs01, 1) * P->max_rhs));
        sl.h01 = tmp;
        P->slots.push_back(sl);
    }
    P->grid = P->slots[0].grid;
    P->grid2 = P->slots[0].grid2;
    P->h0 = P->slots[0].h0;
    P->h1 = P->slots[0].h1;
    P->h01 = P->slots[0].h01;
    if (d == 2) {
        const int nt = g.ntile[0] * g.ntile[1];
        P->spwork.chunk = 128;
        P->spwork.cap = (int)(nt + N / P->spwork.chunk + 1);
        LTRY(P->alloc(&P->spwork.nchunk, nt));
        LTRY(P->alloc(&P->spwork.items, P->spwork.cap));
        LTRY(P->alloc(&P->spwork.total, 1));
        LTRY(P->alloc(&P->sp_offs, nt));
        LTRY(P->alloc(&P->sp_bsum, scan_blocksum_len(nt)));
    }
    // right-hand sides per spreading pass: 1-D a cap on the kernel's chunk (1, 2, 4 or 8), 2-D the
    // chunk itself, as many as the LDS tile holds; the autotuner may lower either
    P->rchunk = g.d == 1 ? 8 : spread_rhs_chunk(g);
    LTRY(P->alloc(&P->B64, (int64_t)T * N));
    if (P->prec == INFFT_F32) LTRY(P->alloc(&P->B32, (int64_t)T * N));
    LTRY(P->alloc(&P->lists, 2 * g.G));
    LTRY(P->alloc(&P->lcount, 8));   // list counters of the solver tiers
    // records: one per block of each solve tier (first tier G/128 blocks at most, the others capped)
    LTRY(P->alloc(&P->stat_rec, (g.G / 64 + 8192) * 5));
    // buffer of the autotuner: max_rhs coefficient vectors or sample vectors, whichever is longer
    {
        char* tmp = nullptr;
        LTRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(g.P, N) * P->max_rhs));
        P->tune_buf = tmp;
    }
    if (P->ws_mode) {
        // workspace plans: everything later calls need is placed now
        LTRY(P->alloc(&P->big_n, g.G));
        for (BigSched& bs : P->big_sched) {
            LTRY(P->alloc(&bs.slot, g.G));
            LTRY(P->alloc(&bs.flag, 2));
        }
        const int64_t lb = (int64_t)(S.o.large_mib > 0 ? S.o.large_mib : 256) << 20;
        char* tmp = nullptr;
        LTRY(P->alloc(&tmp, lb));
        P->large_arena = tmp;
        P->large_arena_bytes = lb;
        if (S.o.ansatz1) {
            LTRY(P->alloc(&P->a1_buf, a1_work_elems(g)));
            P->a1_cap = a1_work_elems(g);
            PlanSpec in1{}, in2{};
            const InnerSpec s1 = a1_symbol_spec(g);
            LTRY(plan_validate(1, &s1.M, s1.N, s1.sigma, s1.m, &s1.o, in1));
            size_t b1 = 0;
            LTRY(plan_measure(in1, &b1));
            LTRY(P->alloc(&tmp, (int64_t)b1));
            P->a1_ws[0] = tmp;
            P->a1_ws_bytes[0] = b1;
            if (P->prec != INFFT_F64) {
                const InnerSpec s2 = a1_twin_spec(g, S.sigma, P->inv_kernel);
                LTRY(plan_validate(1, &s2.M, s2.N, s2.sigma, s2.m, &s2.o, in2));
                size_t b2 = 0;
                LTRY(plan_measure(in2, &b2));
                LTRY(P->alloc(&tmp, (int64_t)b2));
                P->a1_ws[1] = tmp;
                P->a1_ws_bytes[1] = b2;
            }
        }
    }
#undef LTRY
    return INFFT_OK;
}

// Fills the node-independent tables (deconvolution factors, kernel Taylor tables, twiddles, window
// polynomials), reads the ridge's scale and runs the node preprocessing for x.
int plan_setup(infft_plan_s* P, const PlanSpec& S, const double* x) {
    const Geo& g = P->g;
    const int d = g.d, m = g.m;
    int rc;
    for (int t = 0; t < d; ++t) {
        launch_deconv_table(g.M[t], g.Ms[t], m, g.b, P->D64[t], P->D32[t], P->stream);
        if (P->inv_kernel == INFFT_KERNEL_DIRICHLET) {
            std::vector<double> h64(g.M[t], 1.0 / (double)g.Ms[t]);
            h64[0] = 0.0;   // k = -M/2
            std::vector<float> h32(h64.begin(), h64.end());
            HIP_TRY(hipMemcpy(P->Di64[t], h64.data(), sizeof(double) * g.M[t], hipMemcpyHostToDevice));
            if (P->prec == INFFT_F32)
                HIP_TRY(hipMemcpy(P->Di32[t], h32.data(), sizeof(float) * g.M[t], hipMemcpyHostToDevice));
        }
        launch_taylor_table(g.M[t], g.Ms[t], P->Di64[t], 1, P->qK, P->Ktab[t], P->stream);
        launch_taylor_table(g.M[t], g.Ms[t], P->Di64[t], 2, P->qQ, P->Qtab[t], P->stream);
        if (hipGetLastError() != hipSuccess) return fail(INFFT_EDEVICE, "table kernels failed to launch");
    }
    if (d == 1) {
        launch_taylor_table_sym(g.M[0], g.Ms[0], P->Di64[0], 1, P->qK, P->Kstab, P->stream);
        launch_taylor_table_sym(g.M[0], g.Ms[0], P->Di64[0], 2, P->qQ, P->Qstab, P->stream);
        if (hipGetLastError() != hipSuccess) return fail(INFFT_EDEVICE, "table kernels failed to launch");
    }
    for (const TwTable& t : P->tw) launch_twiddles(t.n, t.t64, t.t32, P->stream);
    if (P->split_lo.t64) {
        const int64_t Ms = g.Ms[0], Bsz = P->split_lo.n;
        const int64_t nhi = (Ms + Bsz - 1) / Bsz;
        launch_twiddles_strided(Ms, Bsz, 1, P->split_lo.t64, P->split_lo.t32, P->stream);
        launch_twiddles_strided(Ms, nhi, Bsz, P->split_hi.t64, P->split_hi.t32, P->stream);
    }
    LAUNCH_CHECK();
    if (P->prec == INFFT_F32) {
        std::vector<float> h(P->wpoly_host.begin(), P->wpoly_host.end());
        if (hipMemcpy((void*)P->g.wpoly, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return fail(INFFT_EDEVICE, "uploading the window polynomials failed");
    } else {
        std::vector<double> h(P->wpoly_host.begin(), P->wpoly_host.end());
        if (hipMemcpy((void*)P->g.wpoly, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return fail(INFFT_EDEVICE, "uploading the window polynomials failed");
    }
    // ridge: lambda = rho * (diagonal of G_l) = rho * prod_t M_sigma_t Q_t(0)
    HIP_TRY(hipStreamSynchronize(P->stream));
    double q0 = 1.0;
    for (int t = 0; t < d; ++t) {
        double2 v;
        if (hipMemcpy(&v, P->Qtab[t], sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(INFFT_EDEVICE, "reading the kernel table failed");
        q0 *= v.x * (double)g.Ms[t];
    }
    P->lam = P->rho * q0;
    if (d == 1 && hipMemcpy(&P->dM, P->Di64[0], sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(INFFT_EDEVICE, "reading the deconvolution table failed");
    if ((rc = set_nodes_impl(P, x))) return rc;
    if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(INFFT_EDEVICE, "plan set-up failed on the device");
    (void)S;
    return INFFT_OK;
}

infft_plan_s* plan_new(const PlanSpec& S, void* stream) {
    infft_plan_s* P = new infft_plan_s();
    P->g = S.g;
    P->prec = S.o.precision;
    P->max_rhs = S.o.max_rhs;
    P->rho = S.o.rho;
    P->sigma = S.sigma;
    P->stream = (hipStream_t)stream;
    P->inv_kernel = S.o.inverse_kernel;
    return P;
}

// Bytes of device memory a workspace plan of this specification occupies.
int plan_measure(const PlanSpec& S, size_t* bytes) {
    infft_plan_s* P = plan_new(S, nullptr);
    P->ws_mode = true;
    P->measure = true;
    P->ws_size = SIZE_MAX;
    int rc = plan_layout(P, S);
    *bytes = P->ws_used;
    delete P;
    return rc;
}

// A plan on a caller's workspace (or, with workspace == nullptr, on its own allocations).
int static_scratch_init(int device);
int plan_create(infft_plan* out, const PlanSpec& S, const double* x, void* workspace, size_t workspace_bytes,
                void* stream) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int rc0 = static_scratch_init(dev);
    if (rc0) return rc0;
    infft_plan_s* P = plan_new(S, stream);
    P->device = dev;
    if (workspace) {
        P->ws_mode = true;
        P->ws_base = (char*)workspace;
        P->ws_size = workspace_bytes;
    }
    int rc = plan_layout(P, S);
    if (rc == INFFT_OK) rc = plan_setup(P, S, x);
    if (rc) {
        delete P;
        return rc;
    }
    *out = P;
    return INFFT_OK;
}

// ------------------------------------------------------------------ static scratch
// Work buffers of infft_apply_noalloc, for callers that cannot allocate device memory: a file-scope
// device array (each device the library runs on holds its own copy until the process ends).  Host
// code never passes the array's name to a kernel: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current (at the first plan made on
// it) and kept in g_scratch_ptr.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(INFFT_EDEVICE, "device index %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return INFFT_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(INFFT_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return INFFT_OK;
}

}  // namespace

extern "C" {

int nfft_plan(infft_plan* out, int d, const int64_t* M, int64_t N, double sigma, int m, const double* x,
              const infft_options* opts, void* stream) {
    g_err.clear();
    if (!out) return fail(INFFT_EINVAL, "out is null");
    *out = nullptr;
    if (!x) return fail(INFFT_EINVAL, "x is null");
    PlanSpec S;
    int rc = plan_validate(d, M, N, sigma, m, opts, S);
    if (rc) return rc;
    if (S.o.large_mib || S.o.ansatz1) return fail(INFFT_EINVAL, "large_mib and ansatz1 are options of workspace plans");
    return plan_create(out, S, x, nullptr, 0, stream);
}

int nfft_plan_workspace_bytes(int d, const int64_t* M, int64_t N, double sigma, int m, const infft_options* opts,
                              size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(INFFT_EINVAL, "bytes is null");
    *bytes = 0;
    PlanSpec S;
    int rc = plan_validate(d, M, N, sigma, m, opts, S);
    if (rc) return rc;
    return plan_measure(S, bytes);
}

int nfft_plan_ws(infft_plan* out, int d, const int64_t* M, int64_t N, double sigma, int m, const double* x,
                 const infft_options* opts, void* workspace, size_t workspace_bytes, void* stream) {
    g_err.clear();
    if (!out) return fail(INFFT_EINVAL, "out is null");
    *out = nullptr;
    if (!x) return fail(INFFT_EINVAL, "x is null");
    if (!workspace) return fail(INFFT_EINVAL, "workspace is null");
    if ((uintptr_t)workspace % WS_ALIGN) return fail(INFFT_EINVAL, "workspace must be %d-byte aligned", WS_ALIGN);
    PlanSpec S;
    int rc = plan_validate(d, M, N, sigma, m, opts, S);
    if (rc) return rc;
    size_t need = 0;
    if ((rc = plan_measure(S, &need))) return rc;
    if (workspace_bytes < need)
        return fail(INFFT_ENOMEM, "workspace of %zu bytes is smaller than the %zu bytes the plan needs",
                    workspace_bytes, need);
    return plan_create(out, S, x, workspace, workspace_bytes, stream);
}

int nfft_set_nodes(infft_plan p, const double* x) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (!x) return fail(INFFT_EINVAL, "x is null");
    if (p->batch) {
        BatchState& B = *p->batch;
        p->bopt_ready = false;
        for (size_t i = 0; i < B.subs.size(); ++i) {
            int rc = set_nodes_impl(B.subs[i], x + B.Noff[i] * p->g.d);
            if (rc) return rc;
        }
        return INFFT_OK;
    }
    return set_nodes_impl(p, x);
}

int nfft_set_slot(infft_plan p, int slot) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (p->batch) return fail(INFFT_EINVAL, "nfft_set_slot takes a single-problem plan");
    if (slot < 0 || slot >= (int)p->slots.size())
        return fail(INFFT_EINVAL, "slot %d out of range (the plan has %d)", slot, (int)p->slots.size());
    const infft_plan_s::Slot& sl = p->slots[slot];
    p->cur_slot = slot;
    p->grid = sl.grid;
    p->grid2 = sl.grid2;
    p->h0 = sl.h0;
    p->h1 = sl.h1;
    p->h01 = sl.h01;
    return INFFT_OK;
}

int nfft_set_stream(infft_plan p, void* stream) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    p->stream = (hipStream_t)stream;
    if (p->batch)
        for (infft_plan_s* s : p->batch->subs) s->stream = (hipStream_t)stream;
    return INFFT_OK;
}

static const char* cptr(const infft_plan_s* P, const void* base, int64_t elem_off) {
    return (const char*)base + (int64_t)P->csize() * elem_off;
}


int nfft_trafo(infft_plan p, const void* fhat, void* f, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!fhat || !f) return fail(INFFT_EINVAL, "null data pointer");
    if (p->batch) {
        if ((rc = batch_check_rhs(p, nrhs)) || (rc = run_fft_batched(p, p->batch->to_grid, fhat, nullptr, nrhs)))
            return rc;
        return node_batched(p, NB_INTERP, nullptr, f, nullptr, nrhs);
    }
    const Geo& g = p->g;
    grid_holds(p, 0);
    for (int r0 = 0; r0 < nrhs; r0 += p->max_rhs) {
        const int c = std::min(p->max_rhs, nrhs - r0);
        if ((rc = schedule_for(p, c))) return rc;
        if ((rc = run_fft(p, p->to_grid, cptr(p, fhat, r0 * g.P), nullptr))) return rc;
        void* fo = (void*)cptr(p, f, r0 * g.N);
        ProfScope ps(p, INFFT_K_INTERP);
        if (p->prec == INFFT_F32)
            launch_interp<float>(g, p->nd, (const float2*)p->grid, g.G, (float2*)fo, c, p->stream);
        else
            launch_interp<double>(g, p->nd, (const double2*)p->grid, g.G, (double2*)fo, c, p->stream);
        LAUNCH_CHECK();
    }
    if (nrhs <= p->max_rhs) grid_holds(p, nrhs);   // a single chunk: the grid holds all of it
    return INFFT_OK;
}

static int spread_then_coeffs(infft_plan_s* p, const void* f, void* h, int nrhs, bool useB) {
    const Geo& g = p->g;
    int rc;
    for (int r0 = 0; r0 < nrhs; r0 += p->max_rhs) {
        const int c = std::min(p->max_rhs, nrhs - r0);
        if ((rc = schedule_for(p, c))) return rc;
        const void* fi = cptr(p, f, r0 * g.N);
        {
            ProfScope ps(p, INFFT_K_SPREAD);
            if (p->prec == INFFT_F32)
                launch_spread<float>(g, p->nd, (const float2*)fi, useB ? p->B32 : nullptr, (float2*)p->grid, g.G,
                                     (float2*)p->h0, (float2*)p->h1, (float2*)p->h01, p->hrs0, p->hrs1, p->hrs01, c,
                                     p->rchunk, p->spwork, p->stream);
            else
                launch_spread<double>(g, p->nd, (const double2*)fi, useB ? p->B64 : nullptr, (double2*)p->grid, g.G,
                                      (double2*)p->h0, (double2*)p->h1, (double2*)p->h01, p->hrs0, p->hrs1,
                                      p->hrs01, c, p->rchunk, p->spwork, p->stream);
        }
        LAUNCH_CHECK();
        if ((rc = run_fft(p, p->to_coeff, nullptr, (void*)cptr(p, h, r0 * g.P), useB))) return rc;
    }
    return INFFT_OK;
}

int nfft_adjoint(infft_plan p, const void* f, void* h, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!f || !h) return fail(INFFT_EINVAL, "null data pointer");
    grid_holds(p, 0);
    if (p->batch) {
        if ((rc = batch_check_rhs(p, nrhs)) || (rc = node_batched(p, NB_GATHER, f, nullptr, nullptr, nrhs)))
            return rc;
        return run_fft_batched(p, p->batch->to_coeff, nullptr, h, nrhs);
    }
    return spread_then_coeffs(p, f, h, nrhs, false);
}

// Algorithm 3.17 for a single-problem plan into the given copies of B_opt (either may be null).
// keep_record: replay the recorded pass for large problems where one exists, also outside
// capture (the FP64 recompute of an FP32 plan, which must not replace the record that captured
// graphs replay).
static int precompute_impl(infft_plan p, double2* B64, float2* B32, bool keep_record) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(p->stream, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (capturing && !p->big_sched[0].built)
        return fail(INFFT_ESTATE, "infft_precompute_B under graph capture replays the pass for large local "
                    "problems recorded by the last call outside capture, and there is none yet");
    const bool replay = capturing || (keep_record && p->big_sched[0].built);
    // Replaying a record that holds no large problem there is no pass to enqueue: the last tier
    // itself counts a problem it cannot take as oversized and zeroes its column (which is what the
    // replay would do with a problem the record does not hold), so no launch follows it.
    const bool last_in_place = replay && p->big_sched[0].count == 0;
    const Geo& g = p->g;
    const int64_t TN = (int64_t)p->taps() * g.N;
    p->bopt_ready = false;
    p->out_B64 = B64;
    p->out_B32 = B32;
    // no reset launch: the first tier resets statistics record 0, and the tiers clear the list
    // counters that later launches append to once nothing reads them (the first call of a plan
    // starts from zeros)
    if (g.d == 2) {
        // 1-D tiers write every entry of B_opt themselves (zeros where no problem reaches)
        if (B64) launch_fill_bytes0(B64, TN * (int64_t)sizeof(double2), p->stream);
        if (B32) launch_fill_bytes0(B32, TN * (int64_t)sizeof(float2), p->stream);
    }
    const KTabDev kt = plan_ktab(p);
    SolveArgs a{};
    a.B64 = B64;
    a.B32 = B32;
    a.status = p->status;
    a.stat_rec = p->stat_rec;
    a.stat_off = 1;   // record 0: the large-problem guard
    a.rec0 = p->stat_rec;
    int* listA = p->lists;
    int* listB = p->lists + g.G;
    const int* last_list;
    const int* last_count;
    if (g.d == 1) {
        // one thread per problem for small I(l); the rest in groups of 16 lanes with one row per
        // lane, then the wide tier (up to 32 members on 16 lanes with two rows each, up to 64 on a
        // wavefront), then the blocked pass.  (No separate 32-member launch: each tier is a launch
        // on the critical path even when its list is empty.)
        a.in_list = nullptr;
        a.in_count = nullptr;
        a.out_list = listA;
        a.out_count = p->lcount;
        // counters 1 (read by the last call's wide tier) and 2 (by its large-problem pass)
        a.zero0 = p->lcount + 1;
        a.zero1 = p->lcount + 2;
        {
            ProfScope ps(p, INFFT_K_SOLVE);  // the first tier carries nearly all problems
            a.stat_off += launch_solve_thread_1d(g, p->nd, kt, a, p->stream);
        }
        LAUNCH_CHECK();
        a.rec0 = nullptr;
        a.zero0 = a.zero1 = nullptr;
        a.in_list = listA;
        a.in_count = p->lcount;
        a.out_list = listB;
        a.out_count = p->lcount + 1;
        a.stat_off += launch_solve_tier(g, p->nd, kt, a, 16, p->stream);
        LAUNCH_CHECK();
        // 1-D: the wide tier, up to 64 members (also under capture); it clears counter 0, read by
        // the 16-lane tier that has finished, for the next call's thread tier
        a.in_list = listB;
        a.in_count = p->lcount + 1;
        a.out_list = listA;
        a.out_count = p->lcount + 2;
        a.zero0 = p->lcount;
        last_list = listA;
        last_count = p->lcount + 2;
    } else {
        a.in_list = nullptr;
        a.in_count = nullptr;
        a.out_list = listA;
        a.out_count = p->lcount;
        a.zero0 = p->lcount + 1;   // read by the last call's large-problem pass
        {
            ProfScope ps(p, INFFT_K_SOLVE);
            a.stat_off += launch_solve_tier(g, p->nd, kt, a, 16, p->stream);
        }
        LAUNCH_CHECK();
        a.rec0 = nullptr;
        a.zero0 = nullptr;
        a.in_list = listA;
        a.in_count = p->lcount;
        a.out_list = listB;
        a.out_count = p->lcount + 1;
        last_list = listB;
        last_count = p->lcount + 1;
    }
    if (last_in_place) a.out_list = nullptr;
    a.stat_off += launch_solve_tier(g, p->nd, kt, a, g.d == 1 ? 64 : 32, p->stream);
    LAUNCH_CHECK();
    if (g.d == 2) {
        // counter 0, read by the 32-lane tier just launched, is zero again for the next call
        launch_fill_i32(p->lcount, 1, 0, p->stream);
        LAUNCH_CHECK();
    }
    // problems beyond the register tiers: recorded outside graph capture, replayed under it
    int stat_off = a.stat_off;
    if (!last_in_place) {
        int rc = solve_large(p, kt, last_list, last_count, stat_off, nullptr, replay);
        if (rc) return rc;
    }
    p->stat_nrec = stat_off;   // folded into the status block by nfft_plan_status
    p->bopt_kind = 0;
    p->bopt_ready = true;
    return INFFT_OK;
}

int infft_precompute_B(infft_plan p) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (p->batch) return batch_precompute(p);
    return precompute_impl(p, p->prec == INFFT_F32 ? nullptr : p->B64, p->B32, false);
}

// An FP32 plan's B optimisation keeps only the FP32 copy: before the FP64 values are read, the
// same B optimisation (deterministic, so the FP32 copy is their rounding) runs again into B64.
static int ensure_b64(infft_plan p) {
    if (p->batch || p->prec != INFFT_F32 || p->bopt_kind != 0) return INFFT_OK;
    return precompute_impl(p, p->B64, nullptr, true);
}

int infft_precompute_Bstar(infft_plan p) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (p->batch) return fail(INFFT_EINVAL, "infft_precompute_Bstar takes a single-problem plan");
    grid_holds(p, 0, true);
    const Geo& g = p->g;
    if (g.d != 1) return fail(INFFT_EINVAL, "infft_precompute_Bstar is defined for d = 1");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(p->stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(INFFT_ESTATE, "infft_precompute_Bstar cannot run under graph capture");
    int rc;
    const int M = g.M[0], Ms = g.Ms[0], m = g.m;
    const int nd_all = 2 * m + 1;
    hipStream_t s = p->stream;
    if (p->ws_mode && !p->a1_ws[0])
        return fail(INFFT_ESTATE, "a workspace plan needs the ansatz1 option for infft_precompute_Bstar");
    p->bopt_ready = false;
    // inner plans: on their own allocations, or on the parts of a workspace plan's workspace that
    // nfft_plan_ws placed for them
    auto make_inner = [&](const InnerSpec& is, int k, infft_plan* q) {
        if (p->ws_mode)
            return nfft_plan_ws(q, 1, &is.M, is.N, is.sigma, is.m, p->nd.xw, &is.o, p->a1_ws[k], p->a1_ws_bytes[k], s);
        return nfft_plan(q, 1, &is.M, is.N, is.sigma, is.m, p->nd.xw, &is.o, s);
    };
    // Toeplitz symbol P(q), |q| < M: adjoint NFFT of ones at bandwidth 2M, sigma 2 and the largest
    // cut-off (FP64 accuracy whatever the plan's own m and sigma)
    if (!p->a1_pplan) {
        infft_plan q = nullptr;
        if ((rc = make_inner(a1_symbol_spec(g), 0, &q))) return rc;
        p->a1_pplan = q;
    } else if ((rc = set_nodes_impl(p->a1_pplan, p->nd.xw))) {
        return rc;
    }
    // length-M_sigma FFTs in FP64: the plan itself, or an FP64 twin of an FP32 plan
    infft_plan_s* F = p;
    if (p->prec != INFFT_F64) {
        if (!p->a1_fplan) {
            infft_plan q = nullptr;
            if ((rc = make_inner(a1_twin_spec(g, p->sigma, p->inv_kernel), 1, &q))) return rc;
            p->a1_fplan = q;
        }
        F = p->a1_fplan;
    }
    // K on the grid, whole (M_sigma >= 2M - 1: the products' frequencies |q| < M do not alias) or
    // in two half bands (four products per shift)
    const int nb = Ms >= 2 * M - 1 ? 1 : 2;
    const int npair = nb == 1 ? 1 : 4;
    // work arrays (complex128): S [2m+1][Ms]; R_d [npair][2m+1][Ms], which depends only on M, sigma, m
    // and the kernel and is kept; V [2m+1][Ms]; the FFT intermediate [2m+1][Ms]; the products
    // [npair][2m+1][Ms] (first call only); h [2M], bands [2][M], ones [N]
    const int64_t rows = nd_all;
    const int64_t need = a1_work_elems(g);
    const bool fresh = need > p->a1_cap || (p->ws_mode && !p->a1_R_ready);
    if ((rc = p->grow(&p->a1_buf, p->a1_cap, need))) return rc;
    if (fresh) p->a1_R_ready = false;
    double2* S = p->a1_buf;
    double2* Rc = S + rows * Ms;
    double2* V = Rc + npair * rows * Ms;
    double2* tmp = V + rows * Ms;
    double2* prod = tmp + rows * Ms;
    double2* h = prod + npair * rows * Ms;
    double2* bands = h + 2 * (int64_t)M;
    double2* ones = bands + 2 * (int64_t)M;
    launch_status_init(p->status, 1, s);
    std::vector<FftStep> tg, tc, fw, bw;
    if (!p->a1_R_ready) {
        // a = K's band(s) on the grid, F D 1_band with the inverse's D (into V), then
        // R_d = DFT(conj(a^b) a^c(. - d)) / M_sigma for every pair and shift
        double2* a = V;
        launch_a1_bands(bands, M, nb, s);
        LAUNCH_CHECK();
        if ((rc = build_schedule(F, nb, tg, tc))) return rc;
        if ((rc = run_fft(F, tg, bands, nullptr, true, a, tmp))) return rc;
        launch_a1_products(a, prod, Ms, 0, nd_all, npair, 1.0 / (double)Ms, s);
        LAUNCH_CHECK();
        if ((rc = build_plain_fft(F, nd_all, -1, fw))) return rc;
        for (int c = 0; c < npair; ++c)
            if ((rc = run_fft(F, fw, prod + c * rows * Ms, Rc + c * rows * Ms, false, nullptr, tmp))) return rc;
        p->a1_R_ready = true;
    }
    // Toeplitz symbol P(q) at |q| < M: adjoint NFFT of ones at bandwidth 2M
    launch_a1_ones(ones, g.N, s);
    LAUNCH_CHECK();
    if ((rc = nfft_adjoint(p->a1_pplan, ones, h, 1))) return rc;
    // S(., d) = DFT(fold of P R_d)
    launch_a1_fold(Rc, h, V, M, Ms, nd_all, npair, s);
    LAUNCH_CHECK();
    if ((rc = build_plain_fft(F, nd_all, -1, bw))) return rc;
    if ((rc = run_fft(F, bw, V, S, false, nullptr, tmp))) return rc;
    {
        ProfScope ps(p, INFFT_K_SOLVE);
        launch_a1_solve(g, p->nd, S, p->Ktab[0], p->qK, p->rho, p->B64, p->B32, p->status, s);
    }
    LAUNCH_CHECK();
    p->stat_nrec = 0;
    p->bopt_kind = 1;
    p->bopt_ready = true;
    return INFFT_OK;
}

int infft_apply(infft_plan p, const void* f, void* fcheck, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!f || !fcheck) return fail(INFFT_EINVAL, "null data pointer");
    grid_holds(p, 0);
    if (!p->bopt_ready) return fail(INFFT_ESTATE, "infft_apply before infft_precompute_B");
    if (p->batch) {
        if ((rc = batch_check_rhs(p, nrhs)) || (rc = node_batched(p, NB_GATHER_B, f, nullptr, nullptr, nrhs)))
            return rc;
        return run_fft_batched(p, p->batch->to_coeff, nullptr, fcheck, nrhs, true);
    }
    return spread_then_coeffs(p, f, fcheck, nrhs, true);
}

int infft_apply_noalloc(infft_plan p, const void* f, void* fcheck, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!f || !fcheck) return fail(INFFT_EINVAL, "null data pointer");
    if (p->batch) return fail(INFFT_EINVAL, "infft_apply_noalloc takes a single-problem plan");
    if (!p->bopt_ready) return fail(INFFT_ESTATE, "infft_apply_noalloc before infft_precompute_B");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device) return fail(INFFT_EINVAL, "call infft_apply_noalloc with the plan's device (%d) current", p->device);
    char* base = (char*)g_scratch_ptr[dev];
    if (!base) return fail(INFFT_ESTATE, "the static scratch of device %d is not set up", dev);
    // right-hand sides per pass: as many of the plan's max_rhs as two grids and the halos of that
    // many fit into the static scratch
    const Geo& g = p->g;
    const size_t cs = p->csize();
    auto al = [](size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; };
    auto need = [&](int c) {
        return 2 * al(cs * (size_t)g.G * c) + al(cs * (size_t)std::max<int64_t>(p->hrs0, 1) * c) +
               al(cs * (size_t)std::max<int64_t>(p->hrs1, 1) * c) + al(cs * (size_t)std::max<int64_t>(p->hrs01, 1) * c);
    };
    int chunk = p->max_rhs;
    while (chunk > 1 && need(chunk) > STATIC_SCRATCH_BYTES) --chunk;
    if (need(chunk) > STATIC_SCRATCH_BYTES)
        return fail(INFFT_EINVAL, "one right-hand side needs %zu bytes of work buffers; the static scratch holds %zu",
                    need(1), STATIC_SCRATCH_BYTES);
    // the modified adjoint with the plan's work buffers swapped for the static ones during the call
    void* saved[5] = {p->grid, p->grid2, p->h0, p->h1, p->h01};
    const int saved_rhs = p->max_rhs;
    size_t off = 0;
    p->grid = base + off;
    off += al(cs * (size_t)g.G * chunk);
    p->grid2 = base + off;
    off += al(cs * (size_t)g.G * chunk);
    p->h0 = base + off;
    off += al(cs * (size_t)std::max<int64_t>(p->hrs0, 1) * chunk);
    p->h1 = base + off;
    off += al(cs * (size_t)std::max<int64_t>(p->hrs1, 1) * chunk);
    p->h01 = base + off;
    p->max_rhs = chunk;
    rc = spread_then_coeffs(p, f, fcheck, nrhs, true);
    p->grid = saved[0];
    p->grid2 = saved[1];
    p->h0 = saved[2];
    p->h1 = saved[3];
    p->h01 = saved[4];
    p->max_rhs = saved_rhs;
    return rc;
}

int infft_apply_adjoint(infft_plan p, const void* h, void* f, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!h || !f) return fail(INFFT_EINVAL, "null data pointer");
    grid_holds(p, 0);
    if (!p->bopt_ready) return fail(INFFT_ESTATE, "infft_apply_adjoint before infft_precompute_B");
    if (p->batch) {
        if ((rc = batch_check_rhs(p, nrhs)) || (rc = run_fft_batched(p, p->batch->to_grid, h, nullptr, nrhs, true)))
            return rc;
        return node_batched(p, NB_INTERP_B, nullptr, f, nullptr, nrhs);
    }
    const Geo& g = p->g;
    for (int r0 = 0; r0 < nrhs; r0 += p->max_rhs) {
        const int c = std::min(p->max_rhs, nrhs - r0);
        if ((rc = schedule_for(p, c))) return rc;
        if ((rc = run_fft(p, p->to_grid, cptr(p, h, r0 * g.P), nullptr, true))) return rc;
        void* fo = (void*)cptr(p, f, r0 * g.N);
        ProfScope ps(p, INFFT_K_INTERP);
        if (p->prec == INFFT_F32)
            launch_interp_B<float>(g, p->nd, (const float2*)p->grid, g.G, p->B32, (float2*)fo, c, p->stream);
        else
            launch_interp_B<double>(g, p->nd, (const double2*)p->grid, g.G, p->B64, (double2*)fo, c, p->stream);
        LAUNCH_CHECK();
    }
    return INFFT_OK;
}

int nfft_grad_x(infft_plan p, const void* fhat, const void* gradf, double* gradx, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!fhat || !gradf || !gradx) return fail(INFFT_EINVAL, "null data pointer");
    grid_holds(p, 0);
    if (p->batch) {
        if ((rc = batch_check_rhs(p, nrhs)) || (rc = run_fft_batched(p, p->batch->to_grid, fhat, nullptr, nrhs)))
            return rc;
        return node_batched(p, NB_GRAD, gradf, nullptr, gradx, nrhs);
    }
    const Geo& g = p->g;
    for (int r0 = 0; r0 < nrhs; r0 += p->max_rhs) {
        const int c = std::min(p->max_rhs, nrhs - r0);
        if ((rc = schedule_for(p, c))) return rc;
        if ((rc = run_fft(p, p->to_grid, cptr(p, fhat, r0 * g.P), nullptr))) return rc;
        const void* gf = cptr(p, gradf, r0 * g.N);
        ProfScope ps(p, INFFT_K_INTERP);
        if (p->prec == INFFT_F32)
            launch_grad_x<float>(g, p->nd, (const float2*)p->grid, g.G, (const float2*)gf, gradx, c, r0 > 0,
                                 p->stream);
        else
            launch_grad_x<double>(g, p->nd, (const double2*)p->grid, g.G, (const double2*)gf, gradx, c, r0 > 0,
                                  p->stream);
        LAUNCH_CHECK();
    }
    return INFFT_OK;
}

int nfft_grad_x_after_trafo(infft_plan p, const void* gradf, double* gradx, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!gradf || !gradx) return fail(INFFT_EINVAL, "null data pointer");
    if (p->batch) return fail(INFFT_EINVAL, "nfft_grad_x_after_trafo takes a single-problem plan");
    const int held = p->slots[p->cur_slot].trafo_rhs;
    if (held == 0)
        return fail(INFFT_ESTATE, "work slot %d holds no nfft_trafo result (another call wrote its grid since)",
                    p->cur_slot);
    if (held != nrhs) return fail(INFFT_EINVAL, "nrhs %d differs from the last nfft_trafo's %d", nrhs, held);
    const Geo& g = p->g;
    ProfScope ps(p, INFFT_K_INTERP);
    if (p->prec == INFFT_F32)
        launch_grad_x<float>(g, p->nd, (const float2*)p->grid, g.G, (const float2*)gradf, gradx, nrhs, 0, p->stream);
    else
        launch_grad_x<double>(g, p->nd, (const double2*)p->grid, g.G, (const double2*)gradf, gradx, nrhs, 0,
                              p->stream);
    LAUNCH_CHECK();
    return INFFT_OK;
}

int infft_grad_x_bopt(infft_plan p, const void* f, const void* gradfc, double* gradx, int nrhs) {
    int rc = check_rhs(p, nrhs);
    if (rc) return rc;
    if (!f || !gradfc || !gradx) return fail(INFFT_EINVAL, "null data pointer");
    grid_holds(p, 0);
    if (p->batch) return fail(INFFT_ESTATE, "infft_grad_x_bopt takes a single-problem plan");
    if (!p->bopt_ready) return fail(INFFT_ESTATE, "infft_grad_x_bopt before infft_precompute_B");
    if (p->bopt_kind != 0)
        return fail(INFFT_ESTATE, "infft_grad_x_bopt differentiates the B_opt of infft_precompute_B, not of infft_precompute_Bstar");
    // the gradient reads the FP64 B_opt
    if ((rc = ensure_b64(p))) return rc;
    const Geo& g = p->g;
    launch_fill_bytes0(gradx, (int64_t)sizeof(double) * g.N * g.d, p->stream);
    const KTabDev kt = plan_ktab(p);
    int* listA = p->lists;
    int* listB = p->lists + g.G;
    for (int r0 = 0; r0 < nrhs; r0 += p->max_rhs) {
        const int c = std::min(p->max_rhs, nrhs - r0);
        if ((rc = schedule_for(p, c))) return rc;
        // upstream gradient on the grid: F D gfc with the inverse's D
        if ((rc = run_fft(p, p->to_grid, cptr(p, gradfc, r0 * g.P), nullptr, true))) return rc;
        launch_fill_i32(p->lcount, 8, 0, p->stream);
        BoptGradArgs ga{};
        ga.B64 = p->B64;
        ga.grid = p->grid;
        ga.f = cptr(p, f, r0 * g.N);
        ga.nrhs = c;
        ga.gradx = gradx;
        ga.out_list = listA;
        ga.out_count = p->lcount;
        ProfScope ps(p, INFFT_K_SOLVE);
        if (p->prec == INFFT_F32) launch_bopt_grad<float>(g, p->nd, kt, ga, 16, p->stream);
        else launch_bopt_grad<double>(g, p->nd, kt, ga, 16, p->stream);
        LAUNCH_CHECK();
        ga.in_list = listA;
        ga.in_count = p->lcount;
        ga.out_list = listB;
        ga.out_count = p->lcount + 1;
        if (p->prec == INFFT_F32) launch_bopt_grad<float>(g, p->nd, kt, ga, 32, p->stream);
        else launch_bopt_grad<double>(g, p->nd, kt, ga, 32, p->stream);
        LAUNCH_CHECK();
        // problems beyond 32 members: the blocked factorisation, then their gradient
        int unused = 0;
        if ((rc = solve_large(p, kt, listB, p->lcount + 1, unused, &ga))) return rc;
    }
    // the B optimisation expects its list counters at zero
    launch_fill_i32(p->lcount, 8, 0, p->stream);
    LAUNCH_CHECK();
    return INFFT_OK;
}

int infft_get_B(infft_plan p, void* rows) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (!rows) return fail(INFFT_EINVAL, "rows is null");
    if (!p->bopt_ready) return fail(INFFT_ESTATE, "infft_get_B before infft_precompute_B");
    if (p->batch) {
        const BatchState& B = *p->batch;
        for (size_t i = 0; i < B.subs.size(); ++i) {
            const infft_plan_s* s = B.subs[i];
            launch_export_B(s->g, s->nd.perm, s->B64, (double2*)rows + B.Noff[i] * p->taps(), p->stream);
            LAUNCH_CHECK();
        }
        return INFFT_OK;
    }
    int rc = ensure_b64(p);
    if (rc) return rc;
    launch_export_B(p->g, p->nd.perm, p->B64, (double2*)rows, p->stream);
    LAUNCH_CHECK();
    return INFFT_OK;
}

// Serialised B_opt: a header with the plan's parameters, the wrapped nodes in caller order and
// the rows of B_opt in caller order (the layout of infft_get_B).
struct ExportHeader {
    char magic[8];
    int32_t version;
    int32_t d;
    int64_t M[2];
    int64_t N;
    double sigma;
    int32_t m;
    int32_t inverse_kernel;
    int32_t bopt_kind;
    int32_t taps;
    double rho;
};

static_assert(sizeof(ExportHeader) == 72, "the exported header is 72 bytes");

static const char kExportMagic[8] = {'I', 'N', 'F', 'F', 'T', 'B', 'O', 'P'};

static size_t export_bytes(const infft_plan_s* p) {
    return sizeof(ExportHeader) + (size_t)p->g.N * p->g.d * sizeof(double) +
           (size_t)p->g.N * p->taps() * sizeof(double2);
}

int infft_plan_export(infft_plan p, void* host_buf, size_t* bytes) {
    if (!p || !bytes) return fail(INFFT_EINVAL, "null argument");
    if (p->batch) return fail(INFFT_EINVAL, "infft_plan_export takes a single-problem plan");
    const size_t need = export_bytes(p);
    if (!host_buf) {
        *bytes = need;
        return INFFT_OK;
    }
    if (*bytes < need) return fail(INFFT_EINVAL, "buffer of %zu bytes, %zu needed", *bytes, need);
    if (!p->bopt_ready) return fail(INFFT_ESTATE, "infft_plan_export before infft_precompute_B");
    int rc = ensure_b64(p);
    if (rc) return rc;
    const Geo& g = p->g;
    const int T = p->taps();
    ExportHeader h{};
    std::memcpy(h.magic, kExportMagic, 8);
    h.version = 1;
    h.d = g.d;
    h.M[0] = g.M[0];
    h.M[1] = g.d == 2 ? g.M[1] : 0;
    h.N = g.N;
    h.sigma = p->sigma;
    h.m = g.m;
    h.inverse_kernel = p->inv_kernel;
    h.bopt_kind = p->bopt_kind;
    h.taps = T;
    h.rho = p->rho;
    // the caller's buffer is only byte aligned as far as this layout goes: complex entries are
    // handled as pairs of doubles and copied bytewise
    char* out = (char*)host_buf;
    std::memcpy(out, &h, sizeof(h));
    char* xo = out + sizeof(h);
    char* rows = xo + sizeof(double) * g.N * g.d;
    std::vector<double> Bs((size_t)2 * T * g.N), R((size_t)2 * T * g.N);
    std::vector<int> perm(g.N);
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(xo, p->nd.xw, sizeof(double) * g.N * g.d, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(Bs.data(), p->B64, sizeof(double) * Bs.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(perm.data(), p->nd.perm, sizeof(int) * g.N, hipMemcpyDeviceToHost));
    // internal layout [tap][sorted node] -> caller order [node][tap]
    for (int tau = 0; tau < T; ++tau)
        for (int64_t q = 0; q < g.N; ++q) {
            const size_t dst = 2 * ((size_t)perm[q] * T + tau), src = 2 * ((size_t)tau * g.N + q);
            R[dst] = Bs[src];
            R[dst + 1] = Bs[src + 1];
        }
    std::memcpy(rows, R.data(), sizeof(double) * R.size());
    *bytes = need;
    return INFFT_OK;
}

int infft_plan_import(infft_plan p, const void* host_buf, size_t bytes) {
    if (!p || !host_buf) return fail(INFFT_EINVAL, "null argument");
    if (p->batch) return fail(INFFT_EINVAL, "infft_plan_import takes a single-problem plan");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(p->stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(INFFT_ESTATE, "infft_plan_import cannot run under graph capture");
    const Geo& g = p->g;
    const int T = p->taps();
    if (bytes < sizeof(ExportHeader)) return fail(INFFT_EINVAL, "buffer too short for a header");
    ExportHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (std::memcmp(h.magic, kExportMagic, 8) || h.version != 1) return fail(INFFT_EINVAL, "not an exported B_opt");
    if (h.d != g.d || h.M[0] != g.M[0] || (g.d == 2 && h.M[1] != g.M[1]) || h.N != g.N || h.m != g.m ||
        h.sigma != p->sigma || h.inverse_kernel != p->inv_kernel || h.taps != T || h.rho != p->rho ||
        (h.bopt_kind != 0 && h.bopt_kind != 1))
        return fail(INFFT_EINVAL, "the exported B_opt was made for other plan parameters");
    if (bytes < export_bytes(p)) return fail(INFFT_EINVAL, "buffer of %zu bytes, %zu needed", bytes, export_bytes(p));
    // bytewise copies out of the caller's buffer (its layout does not align complex entries)
    const char* xi = (const char*)host_buf + sizeof(h);
    std::vector<double> R((size_t)2 * T * g.N), Bs((size_t)2 * T * g.N);
    std::memcpy(R.data(), xi + sizeof(double) * g.N * g.d, sizeof(double) * R.size());
    // the nodes, staged in B_opt's storage, through the node preprocessing (which is deterministic,
    // so the sorted order and the lists I(l) are those the B_opt was computed on)
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(p->B64, xi, sizeof(double) * g.N * g.d, hipMemcpyHostToDevice));
    int rc = set_nodes_impl(p, (const double*)p->B64);
    if (rc) return rc;
    std::vector<int> perm(g.N);
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(perm.data(), p->nd.perm, sizeof(int) * g.N, hipMemcpyDeviceToHost));
    for (int tau = 0; tau < T; ++tau)
        for (int64_t q = 0; q < g.N; ++q) {
            const size_t dst = 2 * ((size_t)tau * g.N + q), src = 2 * ((size_t)perm[q] * T + tau);
            Bs[dst] = R[src];
            Bs[dst + 1] = R[src + 1];
        }
    HIP_TRY(hipMemcpy(p->B64, Bs.data(), sizeof(double) * Bs.size(), hipMemcpyHostToDevice));
    if (p->B32) {
        std::vector<float> b32(Bs.size());
        for (size_t i = 0; i < Bs.size(); ++i) b32[i] = (float)Bs[i];
        HIP_TRY(hipMemcpy(p->B32, b32.data(), sizeof(float) * b32.size(), hipMemcpyHostToDevice));
    }
    launch_status_init(p->status, 1, p->stream);
    LAUNCH_CHECK();
    p->stat_nrec = 0;
    p->bopt_kind = h.bopt_kind;
    p->bopt_ready = true;
    return INFFT_OK;
}

int nfft_plan_status(infft_plan p, infft_status* out) {
    if (!p || !out) return fail(INFFT_EINVAL, "null argument");
    if (p->batch) {
        // sums and extremes over the problems of the batch
        std::memset(out, 0, sizeof(*out));
        int64_t mn = INT64_MAX;
        for (infft_plan_s* s : p->batch->subs) {
            infft_status o{};
            int rc = nfft_plan_status(s, &o);
            if (rc && rc != INFFT_ESINGULAR) return rc;
            out->nonfinite_nodes += o.nonfinite_nodes;
            out->failed_solves += o.failed_solves;
            out->empty_columns += o.empty_columns;
            out->oversized += o.oversized;
            if (o.max_members > 0) mn = std::min<int64_t>(mn, o.min_members);
            out->max_members = std::max(out->max_members, o.max_members);
        }
        out->min_members = mn == INT64_MAX ? 0 : mn;
        out->bopt_ready = p->bopt_ready ? 1 : 0;
        out->max_supported = INT32_MAX;
        if (p->bopt_ready && out->failed_solves > 0)
            return fail(INFFT_ESINGULAR, "%lld local solves met a non-positive pivot", (long long)out->failed_solves);
        return INFFT_OK;
    }
    if (p->bopt_ready && p->stat_nrec > 0) {
        launch_solve_stats(p->stat_rec, p->stat_nrec, p->status, p->stream);
        LAUNCH_CHECK();
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    long long st[STATUS_WORDS];
    HIP_TRY(hipMemcpy(st, p->status, sizeof(st), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->nonfinite_nodes = st[ST_NONFINITE];
    out->failed_solves = st[ST_FAILED];
    out->empty_columns = st[ST_EMPTY];
    out->oversized = st[ST_OVERSIZED];
    out->min_members = st[ST_MIN_N] == LLONG_MAX ? 0 : st[ST_MIN_N];
    out->max_members = st[ST_MAX_N];
    out->bopt_ready = p->bopt_ready ? 1 : 0;
    out->max_supported = INT32_MAX;   // limited only by device memory (16 n^2 bytes)
    if (p->bopt_ready && st[ST_FAILED] > 0)
        return fail(INFFT_ESINGULAR, "%lld local solves met a non-positive pivot", st[ST_FAILED]);
    return INFFT_OK;
}

int64_t nfft_plan_device_bytes(infft_plan p) {
    if (!p) return 0;
    int64_t b = p->bytes;
    if (p->a1_pplan) b += p->a1_pplan->bytes;
    if (p->a1_fplan) b += p->a1_fplan->bytes;
    if (p->batch)
        for (const infft_plan_s* s : p->batch->subs) b += s->bytes;
    return b;
}

int infft_autotune(infft_plan p, int reps) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (p->batch) return INFFT_OK;   // batch launches already pack FFT workgroups as LDS allows
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(p->stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(INFFT_ESTATE, "infft_autotune cannot run under graph capture");
    grid_holds(p, 0, true);
    if (reps < 1) reps = 10;
    const Geo& g = p->g;
    const int R = p->max_rhs;
    if (p->ws_mode) {
        // timing in a graph allocates (the graph's executable form): a workspace plan keeps the
        // default shapes
        p->fft_rows[0][0] = p->fft_rows[0][1] = p->fft_rows[1][0] = p->fft_rows[1][1] = 0;
        return build_schedule(p, R, p->to_grid, p->to_coeff);
    }
    void* tmp = p->tune_buf;   // max_rhs x max(prod(M), N) values, placed with the plan
    const size_t tbytes = (size_t)R * (size_t)std::max<int64_t>(g.P, g.N) * p->csize();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t ts = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return fail(INFFT_EDEVICE, "hipEventCreate / hipStreamCreate failed");
    }
    int rc = INFFT_OK;
    if (hipMemsetAsync(tmp, 0, tbytes, p->stream) != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess)
        rc = fail(INFFT_EDEVICE, "hipMemsetAsync failed");
    const bool f32 = p->prec == INFFT_F32;
    auto launch = [&](const FftStep& st) {
        FftIO io{};
        io.in = st.in_buf == 0 ? tmp : st.in_buf == 1 ? p->grid : p->grid2;
        io.out = st.out_buf == 0 ? tmp : st.out_buf == 1 ? p->grid : p->grid2;
        io.D0 = f32 ? (const void*)p->D32[0] : (const void*)p->D64[0];
        io.D1 = f32 ? (const void*)p->D32[1] : (const void*)p->D64[1];
        io.h0 = p->h0;
        io.h1 = p->h1;
        io.h01 = p->h01;
        io.halo_rs0 = p->hrs0;
        io.halo_rs1 = p->hrs1;
        io.halo_rs01 = p->hrs01;
        if (f32) launch_fft_pass<float>(st.pass, io, g, st.ld, st.st, ts);
        else launch_fft_pass<double>(st.pass, io, g, st.ld, st.st, ts);
    };
    // Each direction is timed as it runs in a HIP graph: its passes in sequence, each consuming the
    // last one's output, `reps` times, captured once and replayed.  Eager launches of passes of a
    // few microseconds are paced by the host, which hid the differences between shapes (the shapes
    // chosen that way were up to a fifth slower in graph replays than the defaults).  Candidates:
    // the default shape (0) and every pair of row counts (1, 2, 4, 8, 16 sub-transforms per
    // workgroup, as far as LDS holds them).
    for (int dir = 0; dir < 2 && rc == INFFT_OK; ++dir) {
        float best = 1e30f;
        int best_r[2] = {0, 0};
        for (int ra = 0; ra <= 16 && rc == INFFT_OK; ra = ra ? 2 * ra : 1) {
            for (int rb = 0; rb <= 16 && rc == INFFT_OK; rb = rb ? 2 * rb : 1) {
                if ((ra == 0) != (rb == 0)) continue;
                p->fft_rows[dir][0] = ra;
                p->fft_rows[dir][1] = rb;
                if ((rc = build_schedule(p, R, p->to_grid, p->to_coeff))) break;
                const std::vector<FftStep>& v = dir == 0 ? p->to_grid : p->to_coeff;
                if (v.empty()) break;
                if (ra) {
                    bool valid = v[0].pass.rows == ra && (ra == 1 || ra <= v[0].pass.nseq);
                    if (v.size() > 1) valid = valid && v[1].pass.rows == rb && (rb == 1 || rb <= v[1].pass.nseq);
                    else valid = valid && rb == 1;
                    if (!valid) continue;
                }
                hipGraph_t graph = nullptr;
                hipGraphExec_t exec = nullptr;
                bool ok = hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    for (int i = 0; i < reps; ++i)
                        for (const FftStep& st : v) launch(st);
                    ok = hipStreamEndCapture(ts, &graph) == hipSuccess && graph;
                }
                ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
                float ms = 0.0f;
                ok = ok && hipGraphLaunch(exec, ts) == hipSuccess;   // warm-up
                ok = ok && hipEventRecord(e0, ts) == hipSuccess;
                for (int i = 0; ok && i < 3; ++i) ok = hipGraphLaunch(exec, ts) == hipSuccess;
                ok = ok && hipEventRecord(e1, ts) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (exec) (void)hipGraphExecDestroy(exec);
                if (graph) (void)hipGraphDestroy(graph);
                if (!ok) {
                    rc = fail(INFFT_EDEVICE, "autotune graph timing failed");
                    break;
                }
                if (ms < best) {
                    best = ms;
                    best_r[0] = ra;
                    best_r[1] = rb;
                }
            }
        }
        p->fft_rows[dir][0] = best_r[0];
        p->fft_rows[dir][1] = best_r[1];
    }
    // Right-hand sides per spreading pass (the adjoint's spreading with window weights, max_rhs
    // right-hand sides from the zeroed buffer, into the plan's grid), timed the same way.
    // Candidates: powers of two up to the default (8 in 1-D, the LDS tile's capacity in 2-D) and
    // max_rhs, and the largest itself.
    const int cmax = std::min(g.d == 1 ? 8 : spread_rhs_chunk(g), R);
    if (R > 1 && rc == INFFT_OK) {
        float best = 1e30f;
        int best_c = p->rchunk;
        for (int c = 1; c <= cmax && rc == INFFT_OK; c = (c * 2 > cmax && c < cmax) ? cmax : 2 * c) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            bool ok = hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                for (int i = 0; i < reps; ++i) {
                    if (f32)
                        launch_spread<float>(g, p->nd, (const float2*)tmp, nullptr, (float2*)p->grid, g.G,
                                             (float2*)p->h0, (float2*)p->h1, (float2*)p->h01, p->hrs0, p->hrs1,
                                             p->hrs01, R, c, p->spwork, ts);
                    else
                        launch_spread<double>(g, p->nd, (const double2*)tmp, nullptr, (double2*)p->grid, g.G,
                                              (double2*)p->h0, (double2*)p->h1, (double2*)p->h01, p->hrs0, p->hrs1,
                                              p->hrs01, R, c, p->spwork, ts);
                }
                ok = hipStreamEndCapture(ts, &graph) == hipSuccess && graph;
            }
            ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipGraphLaunch(exec, ts) == hipSuccess;   // warm-up
            ok = ok && hipEventRecord(e0, ts) == hipSuccess;
            for (int i = 0; ok && i < 3; ++i) ok = hipGraphLaunch(exec, ts) == hipSuccess;
            ok = ok && hipEventRecord(e1, ts) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (!ok) {
                rc = fail(INFFT_EDEVICE, "autotune graph timing failed");
                break;
            }
            if (ms < best) {
                best = ms;
                best_c = c;
            }
            if (c == cmax) break;
        }
        p->rchunk = best_c;
        grid_holds(p, 0, true);   // the timing runs wrote the grid
    }
    (void)hipStreamSynchronize(ts);
    (void)hipStreamDestroy(ts);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == INFFT_OK) rc = build_schedule(p, R, p->to_grid, p->to_coeff);
    return rc;
}

int infft_autotune_rows(infft_plan p, int dir, int step) {
    if (!p || dir < 0 || dir > 1 || step < 0 || step > 1) return -1;
    return p->fft_rows[dir][step];
}

int infft_autotune_rhs_chunk(infft_plan p) {
    if (!p) return -1;
    return p->batch ? 0 : p->rchunk;
}

int nfft_plan_batched(infft_plan* out, int nprob, const int64_t* M, const int64_t* N, double sigma, int m,
                      const double* x, const infft_options* opts, void* stream) {
    if (!out) return fail(INFFT_EINVAL, "out is null");
    *out = nullptr;
    if (nprob < 1) return fail(INFFT_EINVAL, "nprob must be positive");
    if (!M || !N || !x) return fail(INFFT_EINVAL, "null size or node pointer");
    infft_options o;
    if (opts) o = *opts;
    else infft_default_options(&o);
    o.work_slots = 1;   // a batch plan runs its problems through one launch per stage, one slot
    auto* P = new infft_plan_s();
    P->batch = new BatchState();
    P->prec = o.precision;
    P->max_rhs = o.max_rhs;
    P->rho = o.rho;
    P->sigma = sigma;
    P->stream = (hipStream_t)stream;
    BatchState& B = *P->batch;
    int64_t poff = 0, noff = 0, goff = 0;
    for (int i = 0; i < nprob; ++i) {
        infft_plan sub = nullptr;
        int rc = nfft_plan(&sub, 1, &M[i], N[i], sigma, m, x + noff, &o, stream);
        if (rc) {
            const std::string msg = "problem " + std::to_string(i) + ": " + g_err;
            delete P;
            g_err = msg;
            return rc;
        }
        B.subs.push_back(sub);
        B.Poff.push_back(poff);
        B.Noff.push_back(noff);
        poff += M[i];
        noff += N[i];
        goff += sub->g.G;
    }
    B.Ptot = poff;
    B.Ntot = noff;
    P->g = B.subs[0]->g;
    P->g.N = noff;
    P->g.P = poff;
    P->g.G = goff;
    int rc = batch_build(P);
    if (rc) {
        delete P;
        return rc;
    }
    *out = P;
    return INFFT_OK;
}

int infft_profile_begin(infft_plan p, int kernel_class) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (kernel_class < INFFT_K_NODES || kernel_class > INFFT_K_SOLVE) return fail(INFFT_EINVAL, "bad kernel class");
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->ev_used = 0;
    p->prof_class = kernel_class;
    return INFFT_OK;
}

int infft_profile_end(infft_plan p, double* total_ms, int64_t* launches) {
    if (!p || !total_ms || !launches) return fail(INFFT_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(p->stream));
    double tot = 0.0;
    for (size_t i = 0; i + 1 < p->ev_used; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev_pool[i], p->ev_pool[i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(p->ev_used / 2);
    p->prof_class = 0;
    p->ev_used = 0;
    return INFFT_OK;
}

void nfft_plan_destroy(infft_plan p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    delete p;
}

}  // extern "C"
