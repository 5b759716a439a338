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

struct infft_plan_s {
    Geo g{};
    int prec = INFFT_F64;
    int max_rhs = 1;
    double rho = 1e-8;
    double sigma = 2.0;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    int64_t bytes = 0;

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

    double2* B64 = nullptr;
    float2* B32 = nullptr;
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

    // large local problems: sizes, failure flags and one batch of matrices and members,
    // allocated when first needed and grown on demand
    int* big_n = nullptr;
    int* big_fail = nullptr;
    int64_t big_fail_cap = 0;
    double2* big_A = nullptr;
    int64_t big_A_cap = 0;
    int* big_midx = nullptr;
    int* big_mtap = nullptr;
    double2* big_mz = nullptr;
    double2* big_mr = nullptr;
    double2* big_mb = nullptr;
    int64_t big_m_cap = 0;
    BigProb* big_probs = nullptr;
    int64_t big_probs_cap = 0;
    int4* big_tasks = nullptr;
    int64_t big_tasks_cap = 0;

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

    ~infft_plan_s() {
        if (batch) batch_free(batch);
        delete a1_pplan;
        delete a1_fplan;
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
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

int ensure_tw(infft_plan_s* P, int64_t n) {
    if (find_tw(P, n)) return INFFT_OK;
    TwTable t;
    t.n = n;
    int rc = P->alloc(&t.t64, n);
    if (rc) return rc;
    if (P->prec == INFFT_F32 && (rc = P->alloc(&t.t32, n))) return rc;
    launch_twiddles(n, t.t64, t.t32, P->stream);
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
    launch_exclusive_scan(P->counts, P->nd.start, g.G, P->bsum, s);
    launch_scatter_nodes(g, P->nd, P->fill, s);
    launch_cell_sort(g, P->nd, P->counts, P->fill, P->nonfinite, P->status, s);
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

// Local problems with more members than the register tiers hold (list of grid indices and its
// device count from the last tier).  Reads the count and the sizes back to the host, sorts the
// problems by size, packs them into batches whose matrices fit the workspace and runs the
// blocked Cholesky pipeline on each batch; adds one statistics record.
int solve_large(infft_plan_s* p, const KTabDev& kt, const int* list, const int* count_dev, int& stat_off,
                const BoptGradArgs* grad = nullptr) {
    const Geo& g = p->g;
    hipStream_t st = p->stream;
    int count = 0;
    HIP_TRY(hipMemcpyAsync(&count, count_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (count <= 0) return INFFT_OK;
    int rc;
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
    const int nmax = ns[order.front()], nmin = ns[order.back()];
    if ((rc = p->grow(&p->big_fail, p->big_fail_cap, count))) return rc;
    launch_fill_i32(p->big_fail, count, 0, st);
    // workspace of one batch: matrices plus member data (40 bytes per member)
    // batch budget: a quarter of the free device memory, between 1 and 16 GiB.  Every batch runs its
    // block steps in sequence, so fewer, larger batches shorten the chain of dependent launches.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    const int64_t kBudget = std::min<int64_t>(std::max<int64_t>((int64_t)(free_b / 4), (int64_t)1 << 30),
                                              (int64_t)16 << 30);
    const int64_t cap_bytes = std::max<int64_t>(kBudget, (int64_t)nmax * nmax * 16 + (int64_t)nmax * 40 + 4096);
    std::vector<BigProb> probs;
    std::vector<int4> tasks;
    size_t pos = 0;
    while (pos < order.size()) {
        probs.clear();
        int64_t ent = 0, mem = 0;
        while (pos < order.size()) {
            const int q = order[pos];
            const int64_t n = ns[q];
            const int64_t e = (n * n + 31) / 32 * 32;
            if (!probs.empty() && (ent + e) * 16 + (mem + n) * 40 > cap_bytes) break;
            BigProb b{};
            b.l = ls[q];
            b.n = (int)n;
            b.nblk = (int)((n + BIG_NB - 1) / BIG_NB);
            b.id = q;
            b.off = ent;
            b.moff = mem;
            probs.push_back(b);
            ent += e;
            mem += n;
            ++pos;
        }
        const int np = (int)probs.size();
        const int T0 = probs.front().nblk;
        // task lists: Gram tiles, then per block column k the panel and trailing tiles
        tasks.clear();
        std::vector<int64_t> seg;   // [gram, trsm_0, herk_0, trsm_1, herk_1, ...] starts
        seg.push_back(0);
        for (int i = 0; i < np; ++i)
            for (int I = 0; I < probs[i].nblk; ++I)
                for (int J = 0; J <= I; ++J) tasks.push_back(make_int4(i, I, J, 0));
        for (int k = 0; k < T0; ++k) {
            seg.push_back((int64_t)tasks.size());
            for (int i = 0; i < np && probs[i].nblk > k; ++i)
                for (int I = k + 1; I < probs[i].nblk; ++I) tasks.push_back(make_int4(i, I, 0, 0));
            seg.push_back((int64_t)tasks.size());
            for (int i = 0; i < np && probs[i].nblk > k; ++i)
                for (int I = k + 1; I < probs[i].nblk; ++I)
                    for (int J = k + 1; J <= I; ++J) tasks.push_back(make_int4(i, I, J, 0));
        }
        seg.push_back((int64_t)tasks.size());
        // substitution steps (right-looking, one launch per block step): forward (problem, I >= k),
        // backward (problem, J <= k)
        std::vector<int64_t> fseg, bseg;
        if (!grad) {
            for (int k = 0; k < T0; ++k) {
                fseg.push_back((int64_t)tasks.size());
                for (int i = 0; i < np && probs[i].nblk > k; ++i)
                    for (int I = k; I < probs[i].nblk; ++I) tasks.push_back(make_int4(i, I, 0, 0));
            }
            fseg.push_back((int64_t)tasks.size());
            for (int k = 0; k < T0; ++k) {
                bseg.push_back((int64_t)tasks.size());
                for (int i = 0; i < np && probs[i].nblk > k; ++i)
                    for (int J = 0; J <= k; ++J) tasks.push_back(make_int4(i, J, 0, 0));
            }
            bseg.push_back((int64_t)tasks.size());
        }
        if ((rc = p->grow(&p->big_A, p->big_A_cap, std::max<int64_t>(ent, 1)))) return rc;
        if (mem > p->big_m_cap) {
            int64_t c1 = p->big_m_cap, c2 = p->big_m_cap, c3 = p->big_m_cap, c4 = p->big_m_cap,
                    c5 = p->big_m_cap;
            if ((rc = p->grow(&p->big_midx, c1, mem)) || (rc = p->grow(&p->big_mtap, c2, mem)) ||
                (rc = p->grow(&p->big_mz, c3, mem)) || (rc = p->grow(&p->big_mr, c4, mem)) ||
                (rc = p->grow(&p->big_mb, c5, mem)))
                return rc;
            p->big_m_cap = c1;
        }
        if ((rc = p->grow(&p->big_probs, p->big_probs_cap, np))) return rc;
        if ((rc = p->grow(&p->big_tasks, p->big_tasks_cap, std::max<int64_t>((int64_t)tasks.size(), 1)))) return rc;
        HIP_TRY(hipMemcpyAsync(p->big_probs, probs.data(), sizeof(BigProb) * np, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(p->big_tasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice, st));
        BigArgs a{};
        a.probs = p->big_probs;
        a.A = p->big_A;
        a.midx = p->big_midx;
        a.mtap = p->big_mtap;
        a.mz = p->big_mz;
        a.mr = p->big_mr;
        a.mb = p->big_mb;
        a.fail = p->big_fail;
        launch_big_setup(g, p->nd, kt, a, np, st);
        LAUNCH_CHECK();
        launch_big_gram(g, kt, a, p->big_tasks + seg[0], (int)(seg[1] - seg[0]), st);
        LAUNCH_CHECK();
        int active = np;
        for (int k = 0; k < T0; ++k) {
            while (active > 0 && probs[active - 1].nblk <= k) --active;
            launch_big_potrf(a, active, k, st);
            LAUNCH_CHECK();
            const int64_t t0 = seg[1 + 2 * k], t1 = seg[2 + 2 * k], t2 = seg[3 + 2 * k];
            launch_big_trsm(a, p->big_tasks + t0, (int)(t1 - t0), k, st);
            LAUNCH_CHECK();
            launch_big_herk(a, p->big_tasks + t1, (int)(t2 - t1), k, st);
            LAUNCH_CHECK();
        }
        if (grad) {
            launch_big_grad(g, a, kt, *grad, p->nd.perm, np, p->prec == INFFT_F32, st);
        } else {
            for (int k = 0; k < T0; ++k) {
                launch_big_fwd(a, p->big_tasks + fseg[k], (int)(fseg[k + 1] - fseg[k]), k, st);
                LAUNCH_CHECK();
            }
            for (int k = T0 - 1; k >= 0; --k) {
                launch_big_bwd(a, p->big_tasks + bseg[k], (int)(bseg[k + 1] - bseg[k]), k, st);
                LAUNCH_CHECK();
            }
            launch_big_write(g, a, np, p->B64, p->B32, st);
        }
        LAUNCH_CHECK();
        // the host task arrays are reused by the next batch
        HIP_TRY(hipStreamSynchronize(st));
    }
    if (grad) return INFFT_OK;   // the precompute's statistics stay as they are
    launch_big_stats(p->big_fail, count, nmin, nmax, p->stat_rec + (int64_t)stat_off * 5, st);
    LAUNCH_CHECK();
    stat_off += 1;
    return INFFT_OK;
}

}  // namespace

// ------------------------------------------------------------------ many 1-D problems in one plan
// A batch plan owns one ordinary plan per problem (its nodes, grid, tables, B_opt, lists) and
// launch tables that let every stage run for all problems in one launch: per launch an array of
// per-problem arguments ("jobs") and a map workgroup -> (job, block of that job).  Caller arrays
// are problem-major: coefficients [problem][nrhs][M_i], samples [problem][nrhs][N_i].

struct BatchLaunch {
    int ld = 0, st = 0;
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
    // ---- FFT passes, grouped by (step index, load mode, store mode)
    std::vector<FftJob> jobs, jobs_inv;
    std::vector<int2> map;
    for (int dir = 0; dir < 2; ++dir) {
        std::map<std::tuple<int, int, int>, std::vector<int>> groups;
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
                groups[std::make_tuple((int)k, st.ld, st.st)].push_back((int)jobs.size());
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
    // ---- solver tiers: thread per problem, then 16- and 32-lane groups over each problem's lists
    std::vector<SolveJob> sj(5 * (size_t)np);
    for (int i = 0; i < np; ++i) {
        infft_plan_s* sub = B.subs[i];
        SolveJob base{};
        base.g = sub->g;
        base.nd = sub->nd;
        base.kt = plan_ktab(sub);
        base.a.B64 = sub->B64;
        base.a.B32 = sub->B32;
        base.a.status = sub->status;
        base.a.stat_rec = sub->stat_rec;
        int* listA = sub->lists;
        int* listB = sub->lists + sub->g.G;
        SolveJob t0 = base, t1 = base, t2 = base, t3 = base;
        t0.a.out_list = listA;
        t0.a.out_count = sub->lcount;
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
        t2.a.stat_off = B.t1_per_prob[i] + B.tier_blocks;
        t3.a.in_list = listA;
        t3.a.in_count = sub->lcount + 2;
        t3.a.out_list = listB;
        t3.a.out_count = sub->lcount + 3;
        t3.a.stat_off = B.t1_per_prob[i] + 2 * B.tier_blocks;
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
                                      user_out, nrhs, P->stream);
        else
            launch_fft_batched<double>(jobs, B.fft_map + L.map_off, L.nblocks, L.shm, L.ld, L.st, user_in,
                                       user_out, nrhs, P->stream);
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
        B.subs[i]->stat_nrec = B.t1_per_prob[i] + 3 * B.tier_blocks;
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

int nfft_plan(infft_plan* out, int d, const int64_t* M, int64_t N, double sigma, int m, const double* x,
              const infft_options* opts, void* stream) {
    g_err.clear();
    if (!out) return fail(INFFT_EINVAL, "out is null");
    *out = nullptr;
    if (d < 1 || d > 2) return fail(INFFT_EINVAL, "d must be 1 or 2 (got %d)", d);
    if (!M) return fail(INFFT_EINVAL, "M is null");
    if (!x) return fail(INFFT_EINVAL, "x is null");
    if (N <= 0 || N >= (int64_t)1 << 31) return fail(INFFT_EINVAL, "N out of range (%lld)", (long long)N);
    if (m < MIN_M_CUT || m > MAX_M_CUT) return fail(INFFT_EINVAL, "m must be in %d..%d (got %d)", MIN_M_CUT, MAX_M_CUT, m);
    if (!(sigma >= 1.0) || !std::isfinite(sigma)) return fail(INFFT_EINVAL, "sigma must be >= 1");
    infft_options o;
    infft_default_options(&o);
    if (opts) o = *opts;
    if (o.precision != INFFT_F32 && o.precision != INFFT_F64) return fail(INFFT_EINVAL, "bad precision");
    if (o.inverse_kernel != INFFT_KERNEL_WINDOW && o.inverse_kernel != INFFT_KERNEL_DIRICHLET)
        return fail(INFFT_EINVAL, "bad inverse_kernel");
    if (o.max_rhs < 1 || o.max_rhs > 64) return fail(INFFT_EINVAL, "max_rhs must be in 1..64");
    const int nslots = o.work_slots == 0 ? 1 : o.work_slots;
    if (nslots < 1 || nslots > 8) return fail(INFFT_EINVAL, "work_slots must be in 1..8 (got %d)", o.work_slots);
    if (!(o.rho >= 0.0) || !std::isfinite(o.rho)) return fail(INFFT_EINVAL, "rho must be finite and >= 0");

    Geo g{};
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
    int64_t n1_split = 0;
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
            n1_split = best;
        }
    }

    infft_plan_s* P = new infft_plan_s();
    P->g = g;
    P->prec = o.precision;
    P->max_rhs = o.max_rhs;
    P->rho = o.rho;
    P->sigma = sigma;
    P->stream = (hipStream_t)stream;
    P->inv_kernel = o.inverse_kernel;
    int rc = INFFT_OK;
#define TRY(e)                     \
    do {                           \
        if ((rc = (e)) != 0) {     \
            delete P;              \
            return rc;             \
        }                          \
    } while (0)
    const int64_t Nd = N * d;
    const int T = P->taps();
    double* xw = nullptr;
    TRY(P->alloc(&xw, Nd));
    P->nd.xw = xw;
    TRY(P->alloc(&P->nd.l0c, Nd));
    TRY(P->alloc(&P->nd.uc, Nd));
    TRY(P->alloc(&P->nd.key, N));
    TRY(P->alloc(&P->nd.perm, N));
    TRY(P->alloc(&P->nd.l0s, Nd));
    TRY(P->alloc(&P->nd.us, Nd));
    TRY(P->alloc(&P->nd.start, g.G + 1));
    TRY(P->alloc(&P->counts, g.G + 1));
    TRY(P->alloc(&P->nonfinite, prep_blocks(g)));
    TRY(P->alloc(&P->fill, g.G));
    TRY(P->alloc(&P->bsum, scan_blocksum_len(g.G) + 1));
    TRY(P->alloc(&P->status, STATUS_WORDS));
    // deconvolution factors and kernel tables
    P->qK = m * TAY_S + 1;
    P->qQ = 2 * m * TAY_S + 1;
    for (int t = 0; t < d; ++t) {
        TRY(P->alloc(&P->D64[t], g.M[t]));
        if (P->prec == INFFT_F32) TRY(P->alloc(&P->D32[t], g.M[t]));
        TRY(P->alloc(&P->Ktab[t], (int64_t)(P->qK + 1) * TAY_NC));
        TRY(P->alloc(&P->Qtab[t], (int64_t)(P->qQ + 1) * TAY_NC));
        launch_deconv_table(g.M[t], g.Ms[t], m, g.b, P->D64[t], P->D32[t], P->stream);
        if (P->inv_kernel == INFFT_KERNEL_DIRICHLET) {
            std::vector<double> h64(g.M[t], 1.0 / (double)g.Ms[t]);
            h64[0] = 0.0;   // k = -M/2
            std::vector<float> h32(h64.begin(), h64.end());
            TRY(P->alloc(&P->Di64[t], g.M[t]));
            HIP_TRY(hipMemcpy(P->Di64[t], h64.data(), sizeof(double) * g.M[t], hipMemcpyHostToDevice));
            if (P->prec == INFFT_F32) {
                TRY(P->alloc(&P->Di32[t], g.M[t]));
                HIP_TRY(hipMemcpy(P->Di32[t], h32.data(), sizeof(float) * g.M[t], hipMemcpyHostToDevice));
            }
        } else {
            P->Di64[t] = P->D64[t];
            P->Di32[t] = P->D32[t];
        }
        launch_taylor_table(g.M[t], g.Ms[t], P->Di64[t], 1, P->qK, P->Ktab[t], P->stream);
        launch_taylor_table(g.M[t], g.Ms[t], P->Di64[t], 2, P->qQ, P->Qtab[t], P->stream);
        if (hipGetLastError() != hipSuccess) TRY(fail(INFFT_EDEVICE, "table kernels failed to launch"));
    }
    if (d == 1) {
        TRY(P->alloc(&P->Kstab, (int64_t)(P->qK + 1) * TAY_NC));
        TRY(P->alloc(&P->Qstab, (int64_t)(P->qQ + 1) * TAY_NC));
        launch_taylor_table_sym(g.M[0], g.Ms[0], P->Di64[0], 1, P->qK, P->Kstab, P->stream);
        launch_taylor_table_sym(g.M[0], g.Ms[0], P->Di64[0], 2, P->qQ, P->Qstab, P->stream);
        if (hipGetLastError() != hipSuccess) TRY(fail(INFFT_EDEVICE, "table kernels failed to launch"));
    }
    // FFT twiddles
    for (int t = 0; t < d; ++t) {
        if (g.Ms[t] <= cap) {
            TRY(ensure_tw(P, g.Ms[t]));
        } else {
            TRY(ensure_tw(P, n1_split));
            TRY(ensure_tw(P, g.Ms[t] / n1_split));
            int64_t Bsz = 1;   // power of two near sqrt(M_sigma): the split of a twiddle exponent is a shift
            while (Bsz * Bsz < g.Ms[t]) Bsz *= 2;
            P->split_lo.n = Bsz;
            P->split_hi.n = n1_split;  // remembered sub-length of the first pass
            const int64_t nhi = (g.Ms[t] + Bsz - 1) / Bsz;
            TRY(P->alloc(&P->split_lo.t64, Bsz));
            TRY(P->alloc(&P->split_hi.t64, nhi));
            if (P->prec == INFFT_F32) {
                TRY(P->alloc(&P->split_lo.t32, Bsz));
                TRY(P->alloc(&P->split_hi.t32, nhi));
            }
            launch_twiddles_strided(g.Ms[t], Bsz, 1, P->split_lo.t64, P->split_lo.t32, P->stream);
            launch_twiddles_strided(g.Ms[t], nhi, Bsz, P->split_hi.t64, P->split_hi.t32, P->stream);
        }
    }
    // window polynomials
    {
        const int nc = P->prec == INFFT_F32 ? WPoly<float>::NC : WPoly<double>::NC;
        const std::vector<long double> cf = window_poly_coeffs(m, (long double)M_PI * (2.0L - 1.0L / sigma), nc);
        if (P->prec == INFFT_F32) {
            std::vector<float> h(cf.begin(), cf.end());
            float* d = nullptr;
            TRY(P->alloc(&d, (int64_t)h.size()));
            if (hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
                TRY(fail(INFFT_EDEVICE, "uploading the window polynomials failed"));
            P->g.wpoly = d;
        } else {
            std::vector<double> h(cf.begin(), cf.end());
            double* d = nullptr;
            TRY(P->alloc(&d, (int64_t)h.size()));
            if (hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                TRY(fail(INFFT_EDEVICE, "uploading the window polynomials failed"));
            P->g.wpoly = d;
        }
    }
    // grids, halos, B_opt, solver lists
    const size_t cs = P->csize();
    const int64_t ntiles = (int64_t)g.ntile[0] * g.ntile[1];
    const int w2 = 2 * m;
    P->hrs0 = ntiles * w2 * (d == 2 ? g.TS[1] : 1);
    P->hrs1 = d == 2 ? ntiles * g.TS[0] * w2 : 0;
    P->hrs01 = d == 2 ? ntiles * w2 * w2 : 0;
    for (int k = 0; k < nslots; ++k) {
        char* tmp = nullptr;
        infft_plan_s::Slot sl{};
        TRY(P->alloc(&tmp, (int64_t)cs * g.G * P->max_rhs));
        sl.grid = tmp;
        TRY(P->alloc(&tmp, (int64_t)cs * g.G * P->max_rhs));
        sl.grid2 = tmp;
        TRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(P->hrs0, 1) * P->max_rhs));
        sl.h0 = tmp;
        TRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(P->hrs1, 1) * P->max_rhs));
        sl.h1 = tmp;
        TRY(P->alloc(&tmp, (int64_t)cs * std::max<int64_t>(P->hrs01, 1) * P->max_rhs));
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
        TRY(P->alloc(&P->spwork.nchunk, nt));
        TRY(P->alloc(&P->spwork.items, P->spwork.cap));
        TRY(P->alloc(&P->spwork.total, 1));
        TRY(P->alloc(&P->sp_offs, nt));
        TRY(P->alloc(&P->sp_bsum, scan_blocksum_len(nt)));
    }
    P->rchunk = spread_rhs_chunk(g);
    TRY(P->alloc(&P->B64, (int64_t)T * N));
    if (P->prec == INFFT_F32) TRY(P->alloc(&P->B32, (int64_t)T * N));
    TRY(P->alloc(&P->lists, 2 * g.G));
    TRY(P->alloc(&P->lcount, 4));
    // records: one per block of each solve tier (first tier G/128 blocks at most, the others capped)
    TRY(P->alloc(&P->stat_rec, (g.G / 64 + 8192) * 5));
    // ridge: lambda = rho * (diagonal of G_l) = rho * prod_t M_sigma_t Q_t(0)
    HIP_TRY(hipStreamSynchronize(P->stream));
    double q0 = 1.0;
    for (int t = 0; t < d; ++t) {
        double2 v;
        if (hipMemcpy(&v, P->Qtab[t], sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
            TRY(fail(INFFT_EDEVICE, "reading the kernel table failed"));
        q0 *= v.x * (double)g.Ms[t];
    }
    P->lam = P->rho * q0;
    if (d == 1 && hipMemcpy(&P->dM, P->Di64[0], sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        TRY(fail(INFFT_EDEVICE, "reading the deconvolution table failed"));
    TRY(set_nodes_impl(P, x));
    if (hipStreamSynchronize(P->stream) != hipSuccess) TRY(fail(INFFT_EDEVICE, "plan set-up failed on the device"));
#undef TRY
    *out = P;
    return INFFT_OK;
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

int infft_precompute_B(infft_plan p) {
    if (!p) return fail(INFFT_EINVAL, "null plan");
    if (p->batch) return batch_precompute(p);
    // The pass for problems beyond the register tiers reads their sizes back to the host; under
    // graph capture it cannot run, and such problems are counted as oversized (zero columns).
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(p->stream, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    const Geo& g = p->g;
    const int64_t TN = (int64_t)p->taps() * g.N;
    p->bopt_ready = false;
    launch_solve_reset(p->status, p->lcount, p->stream);
    if (g.d == 2) {
        // 1-D tiers write every entry of B_opt themselves (zeros where no problem reaches)
        launch_fill_bytes0(p->B64, TN * (int64_t)sizeof(double2), p->stream);
        if (p->B32) launch_fill_bytes0(p->B32, TN * (int64_t)sizeof(float2), p->stream);
    }
    const KTabDev kt = plan_ktab(p);
    SolveArgs a{};
    a.B64 = p->B64;
    a.B32 = p->B32;
    a.status = p->status;
    a.stat_rec = p->stat_rec;
    a.stat_off = 0;
    int* listA = p->lists;
    int* listB = p->lists + g.G;
    const int* last_list;
    const int* last_count;
    if (g.d == 1) {
        // one thread per problem for small I(l); the rest in groups of 16 lanes, then a wavefront
        // per problem up to 64 members, then the blocked pass.  (No 32-lane tier: each tier is a
        // launch on the critical path even when its list is empty, and problems of 17-32 members
        // are rare at the densities this path is built for; the wavefront tier takes them.)
        a.in_list = nullptr;
        a.in_count = nullptr;
        a.out_list = listA;
        a.out_count = p->lcount;
        {
            ProfScope ps(p, INFFT_K_SOLVE);  // the first tier carries nearly all problems
            a.stat_off += launch_solve_thread_1d(g, p->nd, kt, a, p->stream);
        }
        LAUNCH_CHECK();
        a.in_list = listA;
        a.in_count = p->lcount;
        a.out_list = listB;
        a.out_count = p->lcount + 1;
        a.stat_off += launch_solve_tier(g, p->nd, kt, a, 16, p->stream);
        LAUNCH_CHECK();
        // 1-D: a wavefront per problem up to 64 members (also under capture)
        a.in_list = listB;
        a.in_count = p->lcount + 1;
        a.out_list = listA;
        a.out_count = p->lcount + 2;
        last_list = listA;
        last_count = p->lcount + 2;
    } else {
        a.in_list = nullptr;
        a.in_count = nullptr;
        a.out_list = listA;
        a.out_count = p->lcount;
        {
            ProfScope ps(p, INFFT_K_SOLVE);
            a.stat_off += launch_solve_tier(g, p->nd, kt, a, 16, p->stream);
        }
        LAUNCH_CHECK();
        a.in_list = listA;
        a.in_count = p->lcount;
        a.out_list = listB;
        a.out_count = p->lcount + 1;
        last_list = listB;
        last_count = p->lcount + 1;
    }
    if (capturing) {
        a.out_list = nullptr;
        a.out_count = nullptr;
    }
    a.stat_off += launch_solve_tier(g, p->nd, kt, a, g.d == 1 ? 64 : 32, p->stream);
    LAUNCH_CHECK();
    int stat_off = a.stat_off;
    if (!capturing) {
        int rc = solve_large(p, kt, last_list, last_count, stat_off);
        if (rc) return rc;
    }
    p->stat_nrec = stat_off;   // folded into the status block by nfft_plan_status
    p->bopt_kind = 0;
    p->bopt_ready = true;
    return INFFT_OK;
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
    p->bopt_ready = false;
    // Toeplitz symbol P(q), |q| < M: adjoint NFFT of ones at bandwidth 2M, sigma 2 and the largest
    // cut-off (FP64 accuracy whatever the plan's own m and sigma)
    if (!p->a1_pplan) {
        infft_options o;
        infft_default_options(&o);
        o.precision = INFFT_F64;
        const int64_t M2 = 2 * (int64_t)M;
        const int m2 = std::min<int>(MAX_M_CUT, (int)(2 * M2 - 2) / 2);
        infft_plan q = nullptr;
        if ((rc = nfft_plan(&q, 1, &M2, g.N, 2.0, m2, p->nd.xw, &o, s))) return rc;
        p->a1_pplan = q;
    } else if ((rc = set_nodes_impl(p->a1_pplan, p->nd.xw))) {
        return rc;
    }
    // length-M_sigma FFTs in FP64: the plan itself, or an FP64 twin of an FP32 plan
    infft_plan_s* F = p;
    if (p->prec != INFFT_F64) {
        if (!p->a1_fplan) {
            infft_options o;
            infft_default_options(&o);
            o.precision = INFFT_F64;
            o.inverse_kernel = p->inv_kernel;
            const int64_t Mv = M;
            infft_plan q = nullptr;
            if ((rc = nfft_plan(&q, 1, &Mv, 1, p->sigma, m, p->nd.xw, &o, s))) return rc;
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
    const int64_t need = (rows * (3 + 2 * npair)) * Ms + 4 * (int64_t)M + g.N;
    const bool fresh = need > p->a1_cap;
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
        launch_fill_i32(p->lcount, 4, 0, p->stream);
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
    launch_export_B(p->g, p->nd.perm, p->B64, (double2*)rows, p->stream);
    LAUNCH_CHECK();
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
    const int cap = fft_capacity(p->prec == INFFT_F64);
    const int R = p->max_rhs;
    void* tmp = nullptr;
    const size_t tbytes = (size_t)R * (size_t)g.P * p->csize();
    HIP_TRY(hipMalloc(&tmp, tbytes));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(tmp);
        return fail(INFFT_EDEVICE, "hipEventCreate failed");
    }
    int rc = INFFT_OK;
    if (hipMemsetAsync(tmp, 0, tbytes, p->stream) != hipSuccess) rc = fail(INFFT_EDEVICE, "hipMemsetAsync failed");
    for (int dir = 0; dir < 2 && rc == INFFT_OK; ++dir) {
        for (int k = 0; k < 2 && rc == INFFT_OK; ++k) {
            float best = 1e30f;
            int best_rows = 0;
            for (int rows = 1; rows <= 16 && rc == INFFT_OK; rows *= 2) {
                p->fft_rows[dir][k] = rows;
                if ((rc = build_schedule(p, R, p->to_grid, p->to_coeff))) break;
                const std::vector<FftStep>& v = dir == 0 ? p->to_grid : p->to_coeff;
                if ((int)v.size() <= k) break;
                const FftStep& st = v[k];
                if (st.pass.rows != rows) continue;   // beyond the LDS capacity for this length
                if (rows > 1 && rows > st.pass.nseq) break;
                FftIO io{};
                io.in = st.in_buf == 0 ? tmp : st.in_buf == 1 ? p->grid : p->grid2;
                io.out = st.out_buf == 0 ? tmp : st.out_buf == 1 ? p->grid : p->grid2;
                const bool f32 = p->prec == INFFT_F32;
                io.D0 = f32 ? (const void*)p->D32[0] : (const void*)p->D64[0];
                io.D1 = f32 ? (const void*)p->D32[1] : (const void*)p->D64[1];
                io.h0 = p->h0;
                io.h1 = p->h1;
                io.h01 = p->h01;
                io.halo_rs0 = p->hrs0;
                io.halo_rs1 = p->hrs1;
                io.halo_rs01 = p->hrs01;
                auto launch = [&]() {
                    if (f32) launch_fft_pass<float>(st.pass, io, g, st.ld, st.st, p->stream);
                    else launch_fft_pass<double>(st.pass, io, g, st.ld, st.st, p->stream);
                };
                launch();   // warm-up
                (void)hipEventRecord(e0, p->stream);
                for (int i = 0; i < reps; ++i) launch();
                (void)hipEventRecord(e1, p->stream);
                if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(INFFT_EDEVICE, "autotune launch failed");
                    break;
                }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    best_rows = rows;
                }
            }
            p->fft_rows[dir][k] = best_rows;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(p->stream);
    (void)hipFree(tmp);
    if (rc == INFFT_OK) rc = build_schedule(p, R, p->to_grid, p->to_coeff);
    return rc;
}

int infft_autotune_rows(infft_plan p, int dir, int step) {
    if (!p || dir < 0 || dir > 1 || step < 0 || step > 1) return -1;
    return p->fft_rows[dir][step];
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
