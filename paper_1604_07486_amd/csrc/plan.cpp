// plan.cpp -- host side of libthx: plans (Fig. 1 steps 1-2 plus the symbol
// FFT), execution (steps 3-5), a plan cache for the one-shot calls, and the
// C ABI declared in include/thx.h.  All arithmetic of the conversion runs in
// the kernels of kernels.hip; the host only sizes buffers, computes the
// dozen series coefficients of the Gamma-ratio generator, and launches.
#include "../../include/thx.h"
#include "launch.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

using namespace thx;

namespace {

thread_local int g_last_hip_error = 0;

// internal plan flags (above the public THX_FLAG_* bits)
constexpr uint32_t FLAG_IN_CHAIN = 1u << 30; // a stage of a multi-stage conversion
constexpr uint32_t FLAG_SHORT = 1u << 29;    // a batch's bucket of short members: direct evaluation
thread_local bool g_no_timing = false; // thx_execute_noalloc records no events

struct HipFail {
    hipError_t e;
};

inline void hip_check(hipError_t e)
{
    if (e != hipSuccess) throw HipFail{e};
}
inline void launch_check() { hip_check(hipGetLastError()); }

template <typename T>
T *dalloc(int64_t count)
{
    void *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc(&p, (size_t)count * sizeof(T));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    hip_check(e);
    return (T *)p;
}
inline void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

// (dl)_m / m! for m = 0..nt-1 when dl = -n is a negative integer: (-1)^m C(n, m)
// for m <= n and zero beyond (the integer-difference, banded case).  Returns n.
int64_t fill_banded_symbol(double *tsym_dev, int64_t nt, double dl, hipStream_t s);

int64_t fft_length_for(int64_t n, thx_precision prec);
int64_t next_pow2(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int64_t fill_banded_symbol(double *tsym_dev, int64_t nt, double dl, hipStream_t s)
{
    const int64_t n = (int64_t)(-dl);
    std::vector<double> h((size_t)nt, 0.0);
    double c = 1.0; // C(n, m)
    for (int64_t m = 0; m <= n && m < nt; ++m) {
        h[(size_t)m] = (m & 1) ? -c : c;
        c = c * (double)(n - m) / (double)(m + 1);
    }
    hip_check(hipMemcpyAsync(tsym_dev, h.data(), sizeof(double) * (size_t)nt, hipMemcpyHostToDevice, s));
    hip_check(hipStreamSynchronize(s));
    return n;
}

inline bool neg_integer(double x) { return x < 0 && x == std::floor(x); }

} // namespace

// ---------------------------------------------------------------------------
// Gamma-ratio series coefficients: c_j = -B_{2j+1}(x) / (j (2j+1)),
// x = (1 + a - b)/2, with the Bernoulli polynomial B_n(x) = sum_k C(n,k) B_k x^{n-k}.
// ---------------------------------------------------------------------------
GammaRatio thx::make_gamma_ratio(double a, double b)
{
    static const long double Bn[21] = {1.0L, -0.5L, 1.0L / 6, 0, -1.0L / 30, 0, 1.0L / 42, 0,
                                       -1.0L / 30, 0, 5.0L / 66, 0, -691.0L / 2730, 0, 7.0L / 6, 0,
                                       -3617.0L / 510, 0, 43867.0L / 798, 0, -174611.0L / 330};
    GammaRatio g;
    g.a = a;
    g.b = b;
    g.amb = a - b;
    g.pow_mode = (a - b == -0.5) ? -1 : ((a - b == 0.5) ? 1 : 0);
    const long double x = (1.0L + (long double)a - (long double)b) / 2;
    for (int j = 1; j <= GR_TERMS; ++j) {
        const int n = 2 * j + 1;
        long double bp = 0, binom = 1; // C(n, k)
        for (int k = 0; k <= n; ++k) {
            if (k > 0) binom = binom * (long double)(n - k + 1) / (long double)k;
            if (k <= 20 && Bn[k] != 0) bp += binom * Bn[k] * powl(x, (long double)(n - k));
        }
        g.c[j - 1] = (double)(-bp / ((long double)j * (long double)n));
    }
    return g;
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
// One Jacobi conversion stage (a, b) -> (g, b) with the second parameter fixed
// (Sec. 5.3, case 2); `reflect` realises a change of the second parameter as
// R A R, `cheb` folds the Chebyshev normalisation into D1 (1) or D2 (2).
struct JacStage {
    double a = 0, b = 0, g = 0;
    int reflect = 0, cheb = 0;
};
inline bool jac_case3(const JacStage &J) { return !(J.a + J.b > -1.0); }

struct thx_plan {
    thx_kind kind = THX_LEG2CHEB;
    bool is_jac_stage = false;
    bool row0_direct = false; // row 0 by a direct dot product (Hankel PSD on indices >= 1 only)
    JacStage jac;
    thx_plan *next = nullptr; // next stage of a multi-stage conversion
    double *tmp = nullptr;    // intermediate coefficients between stages (ping-pong pair
    double *tmp2 = nullptr;   // for chains of three or more), owned by the first stage
    int64_t tmp_elems = 0;
    double params[4] = {0, 0, 0, 0};
    int64_t N = 0;
    double tol = 0;
    thx_precision prec = THX_FP64;
    uint32_t flags = 0;
    KindDesc kd{};
    int path = 0;   // 0 direct, 1 LDS, 2 three-pass, 3 dense, 4 unit step (suffix sums)
    double *dense = nullptr; // path 3 (reported): At[k][j] = A[j][k], stride dense_ld; the
    int64_t dense_ld = 0;    // stages keep their own path for re-tuning
    uint16_t *dense_bf = nullptr; // FP32-bulk: At split into three bfloat16 parts
    // launch shapes (workgroups targeted per launch), set by the autotuner
    int lds_blocks = 512;    // single-workgroup path: slot groups x vectors
    int lds_radix = 8;       // single-workgroup path: largest FFT radix (8 or 16)
    int p3_blocks = 1024;    // inverse column pass: column tiles x slot groups x vectors
    int p1_blocks = 0;       // forward column pass: column tiles x slot groups x vectors
                             // (0: one workgroup per tile, slot and vector)
    bool fuse_p1 = false;    // columns of 2 or 4: forward column pass fused into the row pass
    int64_t nc = 0;  // complex lanes
    int64_t ncs = 0; // lane stride of the Cholesky columns, packed input and partial sums:
                     // nc rounded up to 128 bytes so that column tiles never straddle lines
    int parts = 0;
    int64_t npart[2] = {0, 0}, a0[2] = {0, 0};
    int64_t L = 0;
    MultiPassGeom geom{};
    int K[2] = {-1, -1};
    double dfinal[2] = {0, 0}; // largest weighted residual at termination / largest weighted diagonal
    double eps[2] = {0, 0};    // stopping threshold in the same units
    double escale[2] = {1, 1}; // converts those units to the API tolerance (thx_plan_achieved_tol)
    int S = 0;            // complex FFT slots
    int slots_alloc = 0;  // allocated slots in ell64
    bool tol_reached = true;
    // device tables
    double *tsym = nullptr;
    double *hk = nullptr;
    bool tsym_alias = false;
    double *d1tab = nullptr, *d2tab = nullptr;
    double *ell64 = nullptr;
    float *ell32 = nullptr;
    double *alias = nullptr; // [2] plan constants of the circulant alias correction
    void *that = nullptr;     // symbol spectrum in working precision (natural or permuted)
    void *twL = nullptr;      // LDS path: w_L^k, k < L
    void *twL1 = nullptr, *twL2 = nullptr, *twA = nullptr; // three-pass tables
    double *tw64_keep[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *pivots[2] = {nullptr, nullptr}; // host copies
    std::vector<double> prel[2];             // weighted pivot value / largest weighted diagonal, per rank
    int S_full = 0; // slots of the whole factorisation (S: those run in this plan's precision)
    // THX_FP64_TAIL32: the trailing slots, whose pivots are so small that single
    // precision rounds them below the Hankel tolerance, run as a single-precision
    // plan of their own (same Cholesky columns, symbol and length); its partial
    // sums join this plan's in the final step
    bool tail_req = false;
    bool tail_on = false;
    thx_plan *tail = nullptr;
    // workspace (grown on demand; executions of one plan must be serialised)
    int64_t ws_batch = 0;
    void *X = nullptr, *Wp = nullptr, *U = nullptr;
    double *row0 = nullptr;
    double *row0_part = nullptr; // [batch][ROW0_PMAX] partial sums of row 0
    double *sfx_tot = nullptr;   // path 4: sub-chunk totals (suffix_tot_doubles)
    int64_t U_slots = 0;
    int Gmax = 0;
    int64_t *vl_off = nullptr, *vl_deg = nullptr; // variable-length executions: per-member offsets, degrees
    int64_t vl_count = 0;
    // per-phase event timing
    uint32_t timing = 0; // bit i: phase i is timed
    std::vector<hipEvent_t> ev_pool;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;

    size_t esize() const { return prec == THX_FP64 ? 16 : 8; }
    ~thx_plan()
    {
        dfree(tsym_alias ? nullptr : tsym);
        dfree(hk);
        dfree(d1tab);
        dfree(d2tab);
        dfree(ell64);
        dfree(ell32);
        dfree(alias);
        dfree(that);
        if (prec == THX_FP64) {
            dfree(twL);
            dfree(twL1);
            dfree(twL2);
            dfree(twA);
        } else {
            dfree(twL);
            dfree(twL1);
            dfree(twL2);
            dfree(twA);
            for (double *p : tw64_keep) dfree(p);
        }
        dfree(X);
        dfree(Wp);
        dfree(U);
        dfree(row0);
        dfree(row0_part);
        dfree(sfx_tot);
        dfree(vl_off);
        dfree(vl_deg);
        delete[] pivots[0];
        delete[] pivots[1];
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        dfree(tmp);
        dfree(tmp2);
        dfree(dense);
        dfree(dense_bf);
        delete tail;
        delete next;
    }
};

namespace {

int64_t direct_crossover()
{
    static int64_t v = [] {
        const char *e = getenv("THX_DIRECT_MAX");
        return e ? (int64_t)atoll(e) : (int64_t)512;
    }();
    return v;
}

// Twiddle table w_M^k (k < count) in the plan's working precision.
void *make_twiddles(thx_plan *p, int64_t M, int64_t count, hipStream_t s, int keep_slot)
{
    double *t64 = dalloc<double>(2 * count);
    if (p->prec == THX_FP64) {
        launch_twiddles(t64, nullptr, M, count, s);
        launch_check();
        return t64;
    }
    float *t32 = dalloc<float>(2 * count);
    launch_twiddles(t64, t32, M, count, s);
    launch_check();
    p->tw64_keep[keep_slot] = t64;
    return t32;
}

// Circulant length for a Toeplitz product of n lanes: the smallest of 2^k,
// 3 * 2^(k-2) and 5 * 2^(k-3) that is >= 2n - 2, the last two only where the
// three-pass path takes them (columns of at least 6 or 10 entries); the
// Toeplitz product is exact for any length >= 2n - 2, and the shorter lengths
// move 3/4 or 5/8 of the bytes (members of mixed batches fall in whichever is
// nearest).  THX_POW2_LENGTHS=1 keeps powers of two.
int64_t fft_length_for(int64_t n, thx_precision prec)
{
    const int64_t need = std::max<int64_t>(64, 2 * n - 2);
    const int64_t p2 = next_pow2(need);
    if (const char *e = getenv("THX_POW2_LENGTHS"))
        if (atoi(e) != 0) return p2;
    const bool f64 = prec != THX_FP32_BULK;
    const int64_t lmax = f64 ? lds_max_len<double>() : lds_max_len<float>();
    const int64_t row = f64 ? mp_row_short<double>() : mp_row_short<float>();
    int64_t best = p2;
    for (const int64_t t : {p2 / 4 * 3, p2 / 8 * 5}) {
        const int64_t min_cols = t % 3 == 0 ? 6 : 10;
        if (t >= need && t < best && t > lmax && t >= min_cols * row && t <= MP_LMAX) best = t;
    }
    return best;
}

// FFT of the embedded symbol in double precision, natural order, scaled by 1/L.
double *symbol_spectrum64(thx_plan *p, hipStream_t s)
{
    const int64_t L = p->L;
    double *emb = dalloc<double>(2 * L);
    double *out = dalloc<double>(2 * L);
    launch_symbol_embed(p->tsym, p->nc, emb, L, s);
    launch_check();
    std::vector<void *> tmp;
    if (L <= lds_max_len<double>()) {
        double *tw = dalloc<double>(2 * L);
        tmp.push_back(tw);
        launch_twiddles(tw, nullptr, L, L, s);
        if (!launch_fft_lds<double>(L, emb, out, tw, 1.0 / (double)L, s)) throw HipFail{hipErrorInvalidValue};
        launch_check();
    } else {
        MultiPassGeom g = multipass_geom<double>(L);
        double *twL1 = dalloc<double>(2 * g.L1), *twL2 = dalloc<double>(2 * g.L2),
               *twA = dalloc<double>(2 * g.L1);
        double *U = dalloc<double>(2 * L), *perm = dalloc<double>(2 * L);
        tmp.insert(tmp.end(), {twL1, twL2, twA, U, perm});
        launch_twiddles(twL1, nullptr, g.L1, g.L1, s);
        launch_twiddles(twL2, nullptr, g.L2, g.L2, s);
        launch_twiddles(twA, nullptr, L, g.L1, s);
        if (!launch_mp_p1<double>(g, nullptr, 0, 0, nullptr, 0, 1, 1, emb, U, 1, twL2, twA, s))
            throw HipFail{hipErrorInvalidValue};
        if (!launch_mp_p2<double>(g, U, 1, 1, nullptr, twL1, twA, twL2, false, perm, 1.0 / (double)L, s))
            throw HipFail{hipErrorInvalidValue};
        // perm[k2 L1 + k1] = spectrum[k2 + L2 k1]  ->  natural order
        launch_reorder<double>(perm, out, L, g.L1, g.L2, 1, s);
        launch_check();
    }
    hip_check(hipStreamSynchronize(s));
    for (void *q : tmp) dfree(q);
    dfree(emb);
    return out;
}

void build_tables(thx_plan *p, hipStream_t s)
{
    const int64_t nt = p->nc, nh = 2 * p->nc + 2;
    if (p->is_jac_stage) {
        // Sec. 5.3 case 2 with b fixed: t_m = (a-g)_m/m!, H_s = Gamma(s+e)/Gamma(s+c+1),
        // e = a+b+1, c = g+b+1; D1, D2 from k_jacobi_diag
        const JacStage &J = p->jac;
        const double dl = J.a - J.g, e = J.a + J.b + 1.0, c = J.g + J.b + 1.0;
        p->tsym = dalloc<double>(nt);
        p->hk = dalloc<double>(nh);
        p->d1tab = dalloc<double>(p->N + 1);
        p->d2tab = dalloc<double>(p->N + 1);
        if (dl == 0.0 || neg_integer(dl)) {
            // identity or integer step (case 1): the Toeplitz factor is banded
            p->kd.band = fill_banded_symbol(p->tsym, nt, dl, s);
        } else {
            launch_gamma_ratio(p->tsym, nt, 0.0, make_gamma_ratio(dl, 1.0), 1.0 / std::tgamma(dl), s);
        }
        launch_gamma_ratio(p->hk, nh, 0.0, make_gamma_ratio(e, c + 1.0), 1.0, s);
        launch_jacobi_diag(p->d1tab, p->N + 1, 1, J.a, J.b, J.g, J.reflect, J.cheb == 1 ? 1 : 0, s);
        launch_jacobi_diag(p->d2tab, p->N + 1, 2, J.a, J.b, J.g, J.reflect, J.cheb == 2 ? 2 : 0, s);
        if (jac_case3(J)) launch_case3_origin(p->hk, p->d1tab, p->d2tab, s);
        p->kd.d1tab = p->d1tab;
        p->kd.d2tab = p->d2tab;
        launch_check();
        return;
    }
    switch (p->kind) {
    case THX_LEG2CHEB: {
        // T_jk = Lambda((k-j)/2), H_jk = Lambda((j+k)/2): one table Lambda(m)
        p->hk = dalloc<double>(nh);
        launch_gamma_ratio(p->hk, nh, 0.0, make_gamma_ratio(0.5, 1.0), 1.0, s);
        p->tsym = p->hk;
        p->tsym_alias = true;
        break;
    }
    case THX_CHEB2LEG: {
        // t_m = Gamma(m - 1/2)/Gamma(m + 1); h(s) = Gamma(s)/Gamma(s + 3/2), h(0) := 1
        p->tsym = dalloc<double>(nt);
        p->hk = dalloc<double>(nh);
        launch_gamma_ratio(p->tsym, nt, 0.0, make_gamma_ratio(-0.5, 1.0), 1.0, s);
        launch_gamma_ratio(p->hk, nh, 0.0, make_gamma_ratio(0.0, 1.5), 1.0, s);
        launch_set_value(p->hk, 1.0, s);
        break;
    }
    case THX_ULTRA2ULTRA: {
        const double l1 = p->params[0], l2 = p->params[1], dl = l1 - l2;
        p->tsym = dalloc<double>(nt);
        p->hk = dalloc<double>(nh);
        // t_m = (dl)_m / m! = Gamma(m + dl) / (Gamma(dl) Gamma(m + 1)); dl = 0 is the
        // identity and a negative integer dl the banded integer step (case 1)
        if (dl == 0.0 || neg_integer(dl)) {
            p->kd.band = 2 * fill_banded_symbol(p->tsym, nt, dl, s); // in units of k - j
        } else {
            launch_gamma_ratio(p->tsym, nt, 0.0, make_gamma_ratio(dl, 1.0), 1.0 / std::tgamma(dl), s);
        }
        // h(s) = (l1)_s / (l2)_{s+1} = Gamma(s + l1) Gamma(l2) / (Gamma(l1) Gamma(s + l2 + 1))
        launch_gamma_ratio(p->hk, nh, 0.0, make_gamma_ratio(l1, l2 + 1.0),
                           std::exp(std::lgamma(l2) - std::lgamma(l1)), s);
        break;
    }
    case THX_LAG2LAG: {
        const double dl = p->params[0] - p->params[1];
        p->tsym = dalloc<double>(nt);
        p->hk = dalloc<double>(nh);
        if (dl == 0.0 || neg_integer(dl)) p->kd.band = fill_banded_symbol(p->tsym, nt, dl, s);
        else launch_gamma_ratio(p->tsym, nt, 0.0, make_gamma_ratio(dl, 1.0), 1.0 / std::tgamma(dl), s);
        // Hankel part = all ones (Sec. 5.4): Gamma(s+1)/Gamma(s+1)
        launch_gamma_ratio(p->hk, nh, 0.0, make_gamma_ratio(1.0, 1.0), 1.0, s);
        break;
    }
    default: throw HipFail{hipErrorInvalidValue};
    }
    launch_check();
}

// Lowest stopping threshold of the pivoted Cholesky, relative to the largest
// weighted diagonal: below a few rounding units of double precision the
// residual diagonal is noise and further pivots would only chase it.
constexpr double PCHOL_FLOOR = 4.440892098500626e-16; // 2^-51

void run_pchol(thx_plan *p, hipStream_t s)
{
    const int64_t maxn = std::max(p->npart[0] - p->a0[0], p->parts == 2 ? p->npart[1] - p->a0[1] : 0);
    int kcap = (int)std::min<int64_t>(KMAX, std::max<int64_t>(maxn, 1));
    p->slots_alloc = p->parts == 2 ? kcap : (kcap + 1) / 2;
    p->ell64 = dalloc<double>(2 * (int64_t)p->slots_alloc * p->ncs);
    hip_check(hipMemsetAsync(p->ell64, 0, sizeof(double) * 2 * (size_t)p->slots_alloc * p->ncs, s));
    double *d = dalloc<double>((int64_t)p->parts * p->ncs);
    double *w = dalloc<double>((int64_t)p->parts * p->ncs);
    PcholState *st = dalloc<PcholState>(1);
    hip_check(hipMemsetAsync(st, 0, sizeof(PcholState), s));
    const int nblk = (int)((p->ncs + 255) / 256);
    double *pv = dalloc<double>((int64_t)p->parts * nblk);
    int *pi = dalloc<int>((int64_t)p->parts * nblk);
    PcholArgs a{};
    a.hk = p->hk;
    a.w = w;
    a.d = d;
    a.ell = p->ell64;
    a.nc = p->ncs;
    for (int q = 0; q < 2; ++q) {
        a.n[q] = p->npart[q];
        a.a0[q] = p->a0[q];
    }
    a.parts = p->parts;
    a.tol = p->tol;
    a.kcap = kcap;
    a.st = st;
    a.pv = pv;
    a.pi = pi;
    a.nblk = nblk;
    launch_pchol_weights(p->kd, a, p->tsym, p->nc, p->tol, PCHOL_FLOOR, s);
    launch_pchol_init(a, s);
    launch_check();
    PcholState hs;
    for (int r = 0; r <= kcap; ++r) {
        launch_pchol_step(a, r, s);
        launch_check();
        if (r % 8 == 7 || r == kcap) {
            int done[2];
            hip_check(hipMemcpyAsync(done, st->done, sizeof(done), hipMemcpyDeviceToHost, s));
            hip_check(hipStreamSynchronize(s));
            bool all = true;
            for (int q = 0; q < p->parts; ++q) all = all && done[q];
            if (all) break;
        }
    }
    hip_check(hipMemcpyAsync(&hs, st, sizeof(PcholState), hipMemcpyDeviceToHost, s));
    hip_check(hipStreamSynchronize(s));
    for (int q = 0; q < p->parts; ++q) {
        p->K[q] = hs.K[q];
        p->dfinal[q] = hs.dfinal[q];
        p->eps[q] = hs.eps[q];
        p->escale[q] = hs.escale[q];
        // not reached: the rank cap came first, or tol lies below the floor
        // (the threshold was raised to it)
        if ((hs.K[q] >= kcap && hs.dfinal[q] > hs.eps[q]) || hs.eps[q] * hs.escale[q] > p->tol * (1 + 1e-12))
            p->tol_reached = false;
        p->pivots[q] = new int32_t[std::max(1, hs.K[q])];
        for (int r = 0; r < hs.K[q]; ++r) p->pivots[q][r] = hs.piv[q][r];
        p->prel[q].resize(std::max(0, hs.K[q]));
        for (int r = 0; r < hs.K[q]; ++r) p->prel[q][r] = hs.dmax0[q] > 0 ? hs.pval[q][r] / hs.dmax0[q] : 0.0;
    }
    p->S = p->parts == 2 ? std::max(p->K[0], p->K[1]) : (p->K[0] + 1) / 2;
    p->S_full = p->S;
    dfree(d);
    dfree(w);
    dfree(st);
    dfree(pv);
    dfree(pi);
}

// ---- FP64 plans with a single-precision tail (THX_FP64_TAIL32) ----
// Slot r's term D_l~r T D_l~r x is of size piv_r / max diag(H) relative to the
// largest (weighted pivots: relative to the largest diagonal entry of A).  Run in single precision, a whole plan whose first pivot is the
// largest diagonal errs by at most 2.7e-8 of ||alpha||_1 (leg2cheb at 2^16 and
// 2^20 with every rank in single precision, measured), so slots whose every
// pivot is at most tol * 2^23 of the largest diagonal add at most ~tol/4
// together, under the truncation the Hankel tolerance already allows
// (2 tol ||alpha||_1 for leg2cheb).
constexpr double TAIL32_PIVOT_GAIN = 8388608.0; // 2^23
constexpr int64_t TAIL32_MIN_L = 8192;             // built from here (single-precision rows of 4096, columns >= 2)
constexpr int64_t TAIL32_ON_L = (int64_t)1 << 16; // on by default from here: shorter single transforms are
                                                  // latency-bound; the autotuner decides for its batch

// first slot from which every later slot has only small pivots
int tail_first_slot(const thx_plan *p)
{
    double gain = TAIL32_PIVOT_GAIN;
    // THX_TAIL32_LOG2GAIN: log2 of the gain (measurements of the error it trades)
    if (const char *e = getenv("THX_TAIL32_LOG2GAIN")) gain = std::ldexp(1.0, atoi(e));
    // pivots within `gain` of the stopping threshold
    auto small = [&](int q, int r) { return r >= p->K[q] || p->prel[q][r] <= p->eps[q] * gain; };
    auto slot_small = [&](int sl) {
        return p->parts == 2 ? small(0, sl) && small(1, sl) : small(0, 2 * sl) && small(0, 2 * sl + 1);
    };
    int s0 = p->S;
    while (s0 > 0 && slot_small(s0 - 1)) --s0;
    return s0;
}

void build_tail(thx_plan *p, const double *spec, hipStream_t s)
{
    if (p->L < TAIL32_MIN_L) return;
    const MultiPassGeom g = multipass_geom<float>(p->L, 0);
    if (!multipass_ok(p->L, g.L1)) return;
    const int s0 = tail_first_slot(p);
    if (s0 >= p->S) return;
    thx_plan *t = new thx_plan();
    p->tail = t; // owned by p from here, also on a later error
    t->kind = p->kind;
    t->kd = p->kd; // device tables stay owned by p
    std::memcpy(t->params, p->params, sizeof(t->params));
    t->N = p->N;
    t->tol = p->tol;
    t->prec = THX_FP32_BULK;
    t->flags = p->flags;
    t->parts = p->parts;
    t->nc = p->nc;
    t->ncs = p->ncs;
    for (int q = 0; q < 2; ++q) {
        t->npart[q] = p->npart[q];
        t->a0[q] = p->a0[q];
    }
    t->L = p->L;
    t->path = 2;
    t->S = t->S_full = p->S - s0;
    t->geom = g;
    t->ell32 = dalloc<float>(2 * (int64_t)t->S * p->ncs);
    launch_cast(p->ell64 + 2 * (int64_t)s0 * p->ncs, t->ell32, 2 * (int64_t)t->S * p->ncs, s);
    launch_check();
    t->twL1 = make_twiddles(t, g.L1, g.L1, s, 0);
    t->twL2 = make_twiddles(t, g.L2, g.L2, s, 1);
    t->twA = make_twiddles(t, p->L, g.L1, s, 2);
    t->that = dalloc<char>((int64_t)t->esize() * p->L);
    launch_reorder<float>(spec, t->that, p->L, g.L1, g.L2, 2, s);
    launch_check();
    p->tail_on = p->L >= TAIL32_ON_L;
    if (p->tail_on) p->S = s0;
}

void build_fft(thx_plan *p, hipStream_t s)
{
    p->L = fft_length_for(p->nc, p->prec);
    if (p->L > ((int64_t)1 << 22)) throw std::invalid_argument("L");
    run_pchol(p, s);
    p->alias = dalloc<double>(2);
    launch_alias_sums(p->ell64, p->ncs, p->S, p->parts, p->L, p->alias, s);
    launch_check();
    const bool f64 = p->prec == THX_FP64;
    if (!f64) {
        p->ell32 = dalloc<float>(2 * (int64_t)std::max(p->S, 1) * p->ncs);
        launch_cast(p->ell64, p->ell32, 2 * (int64_t)p->S * p->ncs, s);
        launch_check();
    }
    double *spec = symbol_spectrum64(p, s); // natural order, scaled by 1/L
    const int64_t L = p->L;
    const int64_t lmax = f64 ? lds_max_len<double>() : lds_max_len<float>();
    if (L <= lmax) {
        p->path = 1;
        // THX_LDS_RADIX: largest FFT radix of this path before any tuning (8 or 16)
        if (const char *e = getenv("THX_LDS_RADIX")) p->lds_radix = atoi(e) == 16 ? 16 : 8;
        p->twL = make_twiddles(p, L, L, s, 0);
        if (f64) {
            p->that = spec;
            spec = nullptr;
        } else {
            p->that = dalloc<char>((int64_t)p->esize() * L);
            launch_reorder<float>(spec, p->that, L, 0, 0, 0, s);
            launch_check();
        }
    } else {
        p->path = 2;
        // THX_ROW_LEN: row length of the three-pass scheme (tuning experiments)
        int64_t row = 0;
        if (const char *e = getenv("THX_ROW_LEN")) row = atoll(e);
        p->geom = f64 ? multipass_geom<double>(L, row) : multipass_geom<float>(L, row);
        // THX_P1_BLOCKS: forward-column-pass workgroups per launch before any tuning
        // (-1: fused into the row pass where the columns allow it)
        if (const char *e = getenv("THX_P1_BLOCKS")) {
            p->p1_blocks = std::max(0, atoi(e));
            p->fuse_p1 = atoi(e) < 0;
        }
        const MultiPassGeom &g = p->geom;
        p->twL1 = make_twiddles(p, g.L1, g.L1, s, 0);
        p->twL2 = make_twiddles(p, g.L2, g.L2, s, 1);
        p->twA = make_twiddles(p, L, g.L1, s, 2);
        // permuted symbol: perm[k2 L1 + k1] = spectrum[k2 + L2 k1]
        p->that = dalloc<char>((int64_t)p->esize() * L);
        if (f64) launch_reorder<double>(spec, p->that, L, g.L1, g.L2, 2, s);
        else launch_reorder<float>(spec, p->that, L, g.L1, g.L2, 2, s);
        launch_check();
        if (p->tail_req) build_tail(p, spec, s);
    }
    dfree(spec);
    hip_check(hipStreamSynchronize(s));
}

thx_status validate_kind(thx_kind kind, const double *params, int nparams, double *out)
{
    auto need = [&](int n) { return nparams >= n && params != nullptr; };
    switch (kind) {
    case THX_LEG2CHEB:
    case THX_CHEB2LEG: return THX_OK;
    case THX_ULTRA2ULTRA: {
        if (!need(2)) return THX_INVALID_ARGUMENT;
        const double l1 = params[0], l2 = params[1];
        if (!(l1 > 0) || !(l2 > 0) || !std::isfinite(l1) || !std::isfinite(l2)) return THX_INVALID_ARGUMENT;
        const double dl = l1 - l2;
        out[0] = l1;
        out[1] = l2;
        // one stage: l1 - l2 <= 1 (case 2; negative integer differences are the
        // banded case 1); larger differences are chained unit steps (case 3)
        (void)dl;
        return THX_OK;
    }
    case THX_JAC2JAC:
    case THX_JAC2CHEB:
    case THX_CHEB2JAC: {
        const int np = kind == THX_JAC2JAC ? 4 : 2;
        if (!need(np)) return THX_INVALID_ARGUMENT;
        for (int i = 0; i < np; ++i) {
            if (!(params[i] > -1) || !std::isfinite(params[i])) return THX_INVALID_ARGUMENT;
            out[i] = params[i];
        }
        return THX_OK;
    }
    case THX_LAG2LAG: {
        if (!need(2)) return THX_INVALID_ARGUMENT;
        const double a1 = params[0], a2 = params[1];
        if (!(a1 > -1) || !(a2 > -1) || !std::isfinite(a1) || !std::isfinite(a2)) return THX_INVALID_ARGUMENT;
        out[0] = a1;
        out[1] = a2;
        return THX_OK;
    }
    default: return THX_UNSUPPORTED;
    }
}

thx_status create_single(thx_plan **out, thx_kind kind, const double *pv, const JacStage *jac, int64_t degree,
                         double tol, thx_precision prec, uint32_t flags, hipStream_t s);

// Link `n` stages made by make(i, &plan) into one plan (the first stage owns the rest).
template <typename Make>
thx_status create_chain(thx_plan **out, size_t n, Make &&make)
{
    thx_plan *first = nullptr, *last = nullptr;
    thx_status r = THX_OK;
    for (size_t i = 0; i < n; ++i) {
        thx_plan *q = nullptr;
        const thx_status ri = make(i, &q);
        if (ri != THX_OK && ri != THX_TOL_NOT_REACHED) {
            delete first;
            return ri;
        }
        if (ri == THX_TOL_NOT_REACHED) r = ri;
        if (last) last->next = q;
        else first = q;
        last = q;
    }
    *out = first;
    return r;
}

// Jacobi conversions (Sec. 5.3): a change of the second parameter b -> d first
// (reflected stage), then of the first a -> g; each stage must be case 2
// (|a - g| < 1 or a - g = 1, and a + b > -1 so that the Hankel part is PSD).
// Level at or below which a fractional Jacobi change between parameters with
// the smaller one `lo` runs (see create_jacobi); THX_JAC_FRAC_LEVEL overrides it
// (measurements of the routes).
double jac_frac_level(double lo)
{
    if (const char *e = getenv("THX_JAC_FRAC_LEVEL")) return (double)atoi(e);
    return lo < 1.0 ? 0.0 : 1.0;
}

thx_status create_jacobi(thx_plan **out, thx_kind kind, const double *pv, int64_t degree, double tol,
                         thx_precision prec, uint32_t flags, hipStream_t s)
{
    double a, b, g, d;
    int cheb_first = 0, cheb_last = 0;
    if (kind == THX_JAC2JAC) {
        a = pv[0], b = pv[1], g = pv[2], d = pv[3];
    } else if (kind == THX_JAC2CHEB) {
        a = pv[0], b = pv[1], g = -0.5, d = -0.5;
        cheb_last = 1;
    } else {
        a = -0.5, b = -0.5, g = pv[0], d = pv[1];
        cheb_first = 2;
    }
    // Sec. 5.3, cases 1 and 4.  A whole-number rise is one banded stage (case 1);
    // a whole-number drop is that many unit steps (T and H constant: suffix sums).
    // A fractional change x -> y runs its case-2 (or case-3) stage at low levels
    // xl = x - kx, yl = y - ky in (lvl - 1, lvl] (so |xl - yl| < 1): kx unit steps
    // down first, the fractional stage, then one banded rise by ky.  Sec. 5.3
    // steps by whole numbers first and takes the fractional stage last; every
    // order gives the same expansion, but the FFT's rounding is relative to the
    // largest term of the whole vector and D1_j ~ j^(g+1) multiplies it, so the
    // fractional stage loses accuracy as its parameters grow, while each unit
    // step down grows the intermediate coefficients.  Measured on the GPU (double
    // precision, degree 3000, error over max_j (|A||alpha|)_j): lvl = 0 is best
    // while min(x, y) < 1 ((0.975 -> 0.847): 1e-15 against 1.4e-12 in place),
    // lvl = 1 above ((1.7 -> 1.2): 3e-14 against 2.6e-12 at lvl 0 and 3.6e-11 at
    // lvl 2; (2.7 -> 2.2): 1.4e-12 against 2.7e-9 at lvl 0).
    std::vector<JacStage> st;
    auto steps = [&](double x, double y, double other, int reflect) {
        if (x == y) return;
        const double dxy = y - x;
        if (dxy == std::floor(dxy)) {
            if (dxy > 0) {
                st.push_back(JacStage{x, other, y, reflect, 0});
            } else {
                for (; x > y; x -= 1.0) st.push_back(JacStage{x, other, x - 1.0, reflect, 0});
            }
            return;
        }
        const double lvl = jac_frac_level(std::min(x, y));
        const double kx = std::max(0.0, std::ceil(x - lvl)), ky = std::max(0.0, std::ceil(y - lvl));
        const double xl = x - kx, yl = y - ky;
        for (; x > xl + 0.5; x -= 1.0) st.push_back(JacStage{x, other, x - 1.0, reflect, 0});
        st.push_back(JacStage{xl, other, yl, reflect, 0});
        if (ky > 0) st.push_back(JacStage{yl, other, y, reflect, 0});
    };
    if (b != d) steps(b, d, a, 1); // (b, a) -> (d, a), reflected
    steps(a, g, d, 0);
    if (st.empty()) st.push_back(JacStage{a, d, g, 0, 0}); // identity (Chebyshev ends still apply)
    st.front().cheb = cheb_first ? cheb_first : st.front().cheb;
    if (cheb_last) {
        if (cheb_first == 0 && st.size() == 1 && st[0].cheb == 0) st[0].cheb = 1;
        else st.back().cheb = 1;
    }
    // case 3 (a + b <= -1) runs with row 0 computed directly, case 1 (integer
    // steps up) with the banded Toeplitz factor
    return create_chain(out, st.size(), [&](size_t i, thx_plan **o) {
        return create_single(o, kind, pv, &st[i], degree, tol, prec, flags | (st.size() > 1 ? FLAG_IN_CHAIN : 0u),
                             s);
    });
}

// ultraspherical, Sec. 5.2 case 3: |lambda1 - lambda2| > 1 (not a whole-number
// rise) moves lambda1 in unit steps towards lambda2, then the remainder (<= 1)
thx_status create_ultra(thx_plan **out, const double *pv, int64_t degree, double tol, thx_precision prec,
                        uint32_t flags, hipStream_t s)
{
    std::vector<std::pair<double, double>> st;
    double l = pv[0];
    while (std::fabs(l - pv[1]) > 1.0 && !(pv[1] > l && neg_integer(l - pv[1]))) {
        const double nl = l > pv[1] ? l - 1.0 : l + 1.0;
        st.push_back({l, nl});
        l = nl;
    }
    st.push_back({l, pv[1]});
    return create_chain(out, st.size(), [&](size_t i, thx_plan **o) {
        const double q[4] = {st[i].first, st[i].second, 0.0, 0.0};
        return create_single(o, THX_ULTRA2ULTRA, q, nullptr, degree, tol, prec,
                             flags | (st.size() > 1 ? FLAG_IN_CHAIN : 0u), s);
    });
}

struct Scratch;
void execute_core(thx_plan *p, const int64_t *off, const int64_t *deg, const double *alpha, double *beta,
                  int64_t degree, int64_t batch, int64_t ld, hipStream_t s, int64_t tmp_elems,
                  const Scratch *sc = nullptr);

// Materialise the matrix of a plan whose stages all run the direct evaluation:
// row k of the identity goes through them and comes out as column k of A, so
// reflections, normalisations, special rows and two-stage products need no
// formulas of their own here.
bool dense_eligible(const thx_plan *p, uint32_t flags)
{
    if (flags & (THX_FLAG_FORCE_FFT | THX_FLAG_NO_DENSE)) return false;
    if (p->N + 1 > DENSE_MAX) return false;
    for (const thx_plan *q = p; q; q = q->next)
        if (q->path != 0) return false;
    return true;
}

void build_dense(thx_plan *p, hipStream_t s)
{
    const int64_t n1 = p->N + 1;
    const int64_t npad = (n1 + DENSE_PAD - 1) / DENSE_PAD * DENSE_PAD;
    double *At = dalloc<double>(npad * npad);
    double *I = nullptr;
    try {
        I = dalloc<double>(n1 * npad);
        launch_zero(At, npad * npad * (int64_t)sizeof(double), s);
        launch_zero(I, n1 * npad * (int64_t)sizeof(double), s);
        launch_identity(I, n1, npad, s);
        execute_core(p, nullptr, nullptr, I, At, p->N, n1, npad, s, n1 * npad);
        hip_check(hipStreamSynchronize(s));
    } catch (...) {
        dfree(I);
        dfree(At);
        throw;
    }
    dfree(I);
    dfree(p->tmp); // the stages' intermediates are not used by the dense product
    dfree(p->tmp2);
    p->tmp = p->tmp2 = nullptr;
    p->tmp_elems = 0;
    p->dense = At;
    p->dense_ld = npad;
    if (p->prec == THX_FP32_BULK) {
        p->dense_bf = dalloc<uint16_t>(dense_bf16_elems(npad));
        launch_split_matrix(At, npad, p->dense_bf, s);
        launch_check();
        hip_check(hipStreamSynchronize(s));
    }
}

void drop_dense(thx_plan *p)
{
    dfree(p->dense);
    dfree(p->dense_bf);
    p->dense = nullptr;
    p->dense_bf = nullptr;
    p->dense_ld = 0;
}

thx_status create_plan(thx_plan **out, thx_kind kind, const double *params, int nparams, int64_t degree,
                       double tol, thx_precision prec, uint32_t flags, hipStream_t s)
{
    if (!out) return THX_INVALID_ARGUMENT;
    *out = nullptr;
    if (degree < 0 || !(tol > 0) || !(tol < 1) ||
        (prec != THX_FP64 && prec != THX_FP32_BULK && prec != THX_FP64_TAIL32))
        return THX_INVALID_ARGUMENT;
    double pv[4] = {0, 0, 0, 0};
    thx_status vs = validate_kind(kind, params, nparams, pv);
    if (vs != THX_OK) return vs;
    thx_status r;
    if (kind == THX_JAC2JAC || kind == THX_JAC2CHEB || kind == THX_CHEB2JAC)
        r = create_jacobi(out, kind, pv, degree, tol, prec, flags, s);
    else if (kind == THX_ULTRA2ULTRA && std::fabs(pv[0] - pv[1]) > 1.0)
        r = create_ultra(out, pv, degree, tol, prec, flags, s);
    else
        r = create_single(out, kind, pv, nullptr, degree, tol, prec, flags, s);
    if ((r != THX_OK && r != THX_TOL_NOT_REACHED) || !dense_eligible(*out, flags)) return r;
    try {
        build_dense(*out, s);
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        delete *out;
        *out = nullptr;
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        delete *out;
        *out = nullptr;
        return THX_OUT_OF_MEMORY;
    }
    return r;
}

thx_status create_single(thx_plan **out, thx_kind kind, const double *pv, const JacStage *jac, int64_t degree,
                         double tol, thx_precision prec, uint32_t flags, hipStream_t s)
{
    thx_plan *p = new (std::nothrow) thx_plan();
    if (!p) return THX_OUT_OF_MEMORY;
    p->kd.band = -1;
    if (jac) {
        p->is_jac_stage = true;
        p->jac = *jac;
    }
    p->kind = kind;
    std::memcpy(p->params, pv, sizeof(p->params));
    p->N = degree;
    p->tol = tol;
    p->prec = prec == THX_FP64_TAIL32 ? THX_FP64 : prec;
    p->tail_req = prec == THX_FP64_TAIL32;
    p->flags = flags;
    p->kd.kind = jac ? (int)THX_JAC2JAC : (int)kind;
    p->kd.parity = (kind == THX_LEG2CHEB || kind == THX_CHEB2LEG || kind == THX_ULTRA2ULTRA) ? 1 : 0;
    for (int i = 0; i < 4; ++i) p->kd.p[i] = pv[i];
    if (p->kd.parity) {
        p->parts = 2;
        p->nc = degree / 2 + 1;
        p->ncs = (p->nc + 15) / 16 * 16;
        p->npart[0] = degree / 2 + 1;
        p->npart[1] = (degree + 1) / 2;
        p->a0[0] = (kind == THX_CHEB2LEG) ? 1 : 0;
        p->a0[1] = 0;
    } else {
        p->parts = 1;
        p->nc = degree + 1;
        p->ncs = (p->nc + 15) / 16 * 16;
        p->npart[0] = degree + 1;
        p->a0[0] = (jac && jac_case3(*jac)) ? 1 : 0;
    }
    p->row0_direct = (kind == THX_CHEB2LEG) || (jac && jac_case3(*jac));
    try {
        build_tables(p, s);
        const bool direct = (flags & (THX_FLAG_FORCE_DIRECT | FLAG_SHORT)) ||
                            (!(flags & THX_FLAG_FORCE_FFT) && degree <= direct_crossover()) ||
                            degree < 2 || p->kd.band >= 0;
        // a parameter lowered by exactly 1: T and H constant (case 1 by suffix sums)
        const bool unit = !p->row0_direct && p->kd.band < 0 &&
                          ((jac && jac->a - jac->g == 1.0) ||
                           ((kind == THX_ULTRA2ULTRA || kind == THX_LAG2LAG) && pv[0] - pv[1] == 1.0));
        // a conversion that is one unit step takes the O(N) suffix sums at every
        // degree (short vectors: one wave each), unless the caller asks for the
        // direct evaluation; inside a chain, short vectors stay direct so that the
        // whole chain can be materialised as one dense matrix
        const bool unit_first = unit && degree >= 2 && !(flags & (FLAG_IN_CHAIN | THX_FLAG_FORCE_DIRECT));
        if (direct && !unit_first) {
            p->path = 0;
            hip_check(hipStreamSynchronize(s));
        } else if (unit) {
            p->path = 4;
            hip_check(hipStreamSynchronize(s));
        } else {
            build_fft(p, s);
        }
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        delete p;
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        delete p;
        return THX_OUT_OF_MEMORY;
    } catch (const std::invalid_argument &) {
        delete p;
        return THX_UNSUPPORTED;
    }
    *out = p;
    return p->tol_reached ? THX_OK : THX_TOL_NOT_REACHED;
}

constexpr size_t MAX_MARKS = 16384;

// Brackets one kernel launch with events when the plan's timing is on.
struct PhaseTimer {
    thx_plan *p;
    hipStream_t s;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    PhaseTimer(thx_plan *p_, int ph, hipStream_t s_) : p(p_), s(s_), phase(ph)
    {
        if (g_no_timing || !((p->timing >> ph) & 1u) || p->marks.size() >= MAX_MARKS) return;
        const size_t need = 2 * (p->marks.size() + 1);
        while (p->ev_pool.size() < need) {
            hipEvent_t e;
            hip_check(hipEventCreate(&e));
            p->ev_pool.push_back(e);
        }
        a = p->ev_pool[need - 2];
        b = p->ev_pool[need - 1];
        hip_check(hipEventRecord(a, s));
    }
    ~PhaseTimer() noexcept(false)
    {
        if (!a) return;
        hip_check(hipEventRecord(b, s));
        p->marks.push_back({phase, a, b});
    }
};

// Workspace of one stage's execution: the plan's own buffers (grown on demand
// by ensure_workspace) or a layout carved from the library's static scratch
// (thx_execute_noalloc).
struct Ws {
    void *X = nullptr, *U = nullptr, *Wp = nullptr;
    double *row0 = nullptr, *row0_part = nullptr, *sfx_tot = nullptr;
    int64_t U_slots = 0;
};
Ws own_ws(const thx_plan *p)
{
    Ws w;
    w.X = p->X;
    w.U = p->U;
    w.Wp = p->Wp;
    w.row0 = p->row0;
    w.row0_part = p->row0_part;
    w.sfx_tot = p->sfx_tot;
    w.U_slots = p->U_slots;
    return w;
}

// Partial-sum groups of an execution of `batch` vectors with slot chunks of
// `us` (the three-pass path) -- the count run_slots produces.
int64_t groups_for(const thx_plan *p, int64_t batch, int64_t us)
{
    if (p->S <= 0) return 1;
    if (p->path == 1) {
        const int64_t Gt = std::min<int64_t>(p->S, std::max<int64_t>(1, (p->lds_blocks + batch - 1) / batch));
        const int64_t spg = (p->S + Gt - 1) / Gt;
        return (p->S + spg - 1) / spg;
    }
    const int64_t tiles = p->geom.L1 / p->geom.TC;
    int64_t G = 0;
    for (int64_t s0 = 0; s0 < p->S; s0 += us) {
        const int64_t ns = std::min<int64_t>(us, p->S - s0);
        int64_t Gc = std::min<int64_t>(ns, std::max<int64_t>(1, (p->p3_blocks + tiles * batch - 1) / (tiles * batch)));
        const int64_t spg = (ns + Gc - 1) / Gc;
        G += (ns + spg - 1) / spg;
    }
    return G;
}

void ensure_workspace(thx_plan *p, int64_t batch)
{
    if (p->tail) ensure_workspace(p->tail, batch);
    if (batch <= p->ws_batch) return;
    if (p->path == 4) {
        dfree(p->sfx_tot);
        p->sfx_tot = nullptr;
        p->ws_batch = 0;
        p->sfx_tot = dalloc<double>(suffix_tot_doubles(p->kd, p->N, batch));
        p->ws_batch = batch;
        return;
    }
    dfree(p->X);
    dfree(p->Wp);
    dfree(p->U);
    dfree(p->row0);
    dfree(p->row0_part);
    p->X = p->Wp = p->U = nullptr;
    p->row0 = nullptr;
    p->row0_part = nullptr;
    p->ws_batch = 0;
    const size_t es = p->esize();
    p->X = dalloc<char>((int64_t)(es * (size_t)(batch * p->ncs)));
    const int slots = std::max(p->S, p->S_full); // the tail may be switched off
    p->Gmax = std::max(1, slots);
    p->Wp = dalloc<char>((int64_t)(es * (size_t)((int64_t)p->Gmax * batch * p->ncs)));
    p->row0 = dalloc<double>(batch);
    if (p->row0_direct) p->row0_part = dalloc<double>(batch * ROW0_PMAX);
    if (p->path == 2) {
        // slot chunk so that the FFT intermediates stay within ~8 GiB (of the
        // 288 GB of HBM): fewer chunks mean fewer launches and fewer partial-sum
        // groups for the final step to read
        const int64_t per = (int64_t)es * p->L * batch;
        int64_t sc = std::max<int64_t>(1, ((int64_t)8 << 30) / per);
        if (const char *e = getenv("THX_SLOT_CHUNK")) sc = std::max<int64_t>(1, std::min<int64_t>(sc, atoll(e)));
        sc = std::min<int64_t>(sc, std::max(1, slots));
        p->U_slots = sc;
        p->U = dalloc<char>(per * sc);
    }
    p->ws_batch = batch;
}

// slots per forward-column-pass workgroup for `ns` slots of `batch` vectors
int p1_slots_per_block(const thx_plan *p, int ns, int64_t batch)
{
    if (p->p1_blocks <= 0) return 1;
    const int64_t items = p->geom.L1 / p->geom.TC * (int64_t)ns * batch;
    return (int)std::max<int64_t>(1, std::min<int64_t>(ns, items / p->p1_blocks));
}

// Pack the vectors and run the plan's slots (single workgroup or three passes)
// into its partial sums; returns the number of partial-sum groups.  Phases are
// timed on `tm` (the plan the caller executes).
template <typename T>
int run_slots(thx_plan *p, const Ws &w, thx_plan *tm, const int64_t *off, const int64_t *deg, const double *alpha,
              int64_t N, int64_t batch, int64_t ld, hipStream_t s)
{
    const int64_t n = p->kd.parity ? N / 2 + 1 : N + 1;
    const void *ell = p->prec == THX_FP64 ? (const void *)p->ell64 : (const void *)p->ell32;
    // For one vector the forward column pass forms its input lanes from the
    // vector itself and the pack launch is skipped: with one slot per workgroup
    // up to L = 2^17 (measured 2 us faster at N = 2^16 in both precisions, and
    // 1.4 us at N = 2048 on the single-workgroup path, which follows the same
    // rule: 15.5 -> 14.1 us), and in double precision with slot groups at any
    // length (each workgroup forms its tile's lanes once for its slots; 2^20
    // 0.770 -> 0.766 ms).  Above 2^17, re-forming the lanes for each of 45
    // slots cost 8 us more than the pack launch at 2^20, and on the
    // 4096-polynomial batch 1.2-1.6 ms more (members at odd offsets take two
    // 8-byte loads per lane in every slot); single-precision lanes are half the
    // bytes of the vector they come from, so slot groups read them packed there
    // (2^22: 1.019 -> 1.02-1.04 ms formed from the vector); batches and the
    // fused row pass read them packed.
    const bool fused = p->path == 2 && p->fuse_p1 && p->geom.L2 <= 4;
    const bool groups = sizeof(T) == 8 && p->path == 2 &&
                        p1_slots_per_block(p, (int)std::min<int64_t>(w.U_slots, p->S), batch) > 1;
    const bool packed = p->S <= 0 || batch != 1 || fused || (p->path != 1 && p->path != 2) ||
                        (p->L > ((int64_t)1 << 17) && !groups);
    const AlphaIn ain{p->kd, off, deg, alpha, ld, N};
    if (packed) {
        PhaseTimer t(tm, THX_PHASE_PACK, s);
        launch_pack<T>(p->kd, off, deg, alpha, ld, N, batch, w.X, p->ncs, s);
    }
    int G = 0;
    if (p->S > 0) {
        if (p->path == 1) {
            int Gt = (int)std::min<int64_t>(p->S, std::max<int64_t>(1, (p->lds_blocks + batch - 1) / batch));
            const int spg = (p->S + Gt - 1) / Gt;
            G = (p->S + spg - 1) / spg;
            PhaseTimer t(tm, THX_PHASE_TOEP_LDS, s);
            if (!launch_toep_lds<T>(p->L, p->lds_radix, packed ? w.X : nullptr, p->ncs, n, ell, p->S, spg, G,
                                    p->that, p->twL, w.Wp, batch, s, packed ? nullptr : &ain))
                throw HipFail{hipErrorInvalidValue};
        } else {
            const MultiPassGeom &g = p->geom;
            const int64_t tiles = g.L1 / g.TC;
            for (int s0 = 0; s0 < p->S; s0 += (int)w.U_slots) {
                const int ns = (int)std::min<int64_t>(w.U_slots, p->S - s0);
                if (p->fuse_p1 && g.L2 <= 4) {
                    PhaseTimer t(tm, THX_PHASE_ROW, s);
                    if (!launch_mp_p2f<T>(g, w.X, p->ncs, n, ell, s0, ns, w.U, batch, p->that, p->twL1, p->twA,
                                          p->twL2, s))
                        throw HipFail{hipErrorInvalidValue};
                } else {
                    {
                        PhaseTimer t(tm, THX_PHASE_COL_FWD, s);
                        if (!launch_mp_p1<T>(g, packed ? w.X : nullptr, p->ncs, n, ell, s0, ns,
                                             p1_slots_per_block(p, ns, batch), nullptr, w.U, batch, p->twL2,
                                             p->twA, s, packed ? nullptr : &ain))
                            throw HipFail{hipErrorInvalidValue};
                    }
                    PhaseTimer t(tm, THX_PHASE_ROW, s);
                    if (!launch_mp_p2<T>(g, w.U, ns, batch, p->that, p->twL1, p->twA, p->twL2, true, nullptr, 1.0, s))
                        throw HipFail{hipErrorInvalidValue};
                }
                int Gc = (int)std::min<int64_t>(
                    ns, std::max<int64_t>(1, (p->p3_blocks + tiles * batch - 1) / (tiles * batch)));
                const int spg = (ns + Gc - 1) / Gc;
                Gc = (ns + spg - 1) / spg;
                {
                    PhaseTimer t(tm, THX_PHASE_COL_INV, s);
                    if (!launch_mp_p3<T>(g, w.U, p->ncs, n, ell, s0, ns, spg, Gc, w.Wp, G, batch, p->twL2, s))
                        throw HipFail{hipErrorInvalidValue};
                }
                G += Gc;
            }
        }
    } else {
        launch_zero(w.Wp, (int64_t)(p->esize() * (size_t)(batch * p->ncs)), s);
        G = 1;
    }
    return G;
}

template <typename T>
void execute_fft(thx_plan *p, const Ws &w, const Ws &wt, const int64_t *off, const int64_t *deg,
                 const double *alpha, double *beta, int64_t N, int64_t batch, int64_t ld, hipStream_t s)
{
    const int G = run_slots<T>(p, w, p, off, deg, alpha, N, batch, ld, s);
    thx_plan *t = p->tail_on ? p->tail : nullptr;
    const int G2 = t ? run_slots<float>(t, wt, p, off, deg, alpha, N, batch, ld, s) : 0;
    const double *row0 = nullptr;
    if (p->row0_direct) {
        PhaseTimer tm(p, THX_PHASE_ROW0, s);
        launch_row0_direct(p->kd, off, deg, alpha, ld, N, batch, p->tsym, p->hk, w.row0_part, w.row0, s);
        row0 = w.row0;
    }
    {
        PhaseTimer tm(p, THX_PHASE_UNPACK, s);
        launch_unpack<T>(p->kd, off, deg, alpha, ld, beta, N, batch, w.Wp, G, t ? wt.Wp : nullptr, G2, p->ncs,
                         p->L, p->alias, p->tsym, row0, s);
    }
    launch_check();
}

// A static scratch region handed to one execution (thx_execute_noalloc):
// intermediates between stages first, then one region every stage reuses in
// turn (the stages run one after another on the stream).
struct Scratch {
    char *base = nullptr;
    int64_t bytes = 0;
    double *tmp = nullptr, *tmp2 = nullptr;
    char *region = nullptr;
    int64_t region_bytes = 0;
};

void execute_stage(thx_plan *p, const int64_t *off, const int64_t *deg, const double *alpha, double *beta,
                   int64_t degree, int64_t batch, int64_t ld, hipStream_t s, const Scratch *sc = nullptr);

void ensure_tmp(thx_plan *p, int64_t elems)
{
    if (elems <= p->tmp_elems) return;
    dfree(p->tmp);
    dfree(p->tmp2);
    p->tmp = p->tmp2 = nullptr;
    p->tmp_elems = 0;
    p->tmp = dalloc<double>(elems);
    if (p->next && p->next->next) p->tmp2 = dalloc<double>(elems);
    p->tmp_elems = elems;
}

// Launch the whole execution on `s` (no host synchronisation, no allocation
// once the workspace is sized, no memset nodes: graph-capturable).  Two-stage
// plans go through the plan's intermediate buffer of `tmp_elems` doubles
// (laid out like alpha).
void execute_core(thx_plan *p, const int64_t *off, const int64_t *deg, const double *alpha, double *beta,
                  int64_t degree, int64_t batch, int64_t ld, hipStream_t s, int64_t tmp_elems, const Scratch *sc)
{
    if (p->dense) {
        PhaseTimer t(p, THX_PHASE_DENSE, s);
        if (p->dense_bf) launch_dense_bf16(p->dense_bf, p->dense_ld, off, deg, alpha, ld, beta, degree, batch, s);
        else launch_dense(p->dense, p->dense_ld, off, deg, alpha, ld, beta, degree, batch, s);
        launch_check();
        return;
    }
    if (!p->next) {
        execute_stage(p, off, deg, alpha, beta, degree, batch, ld, s, sc);
        return;
    }
    if (!sc) ensure_tmp(p, tmp_elems);
    double *bufs[2] = {sc ? sc->tmp : p->tmp, sc ? sc->tmp2 : p->tmp2};
    const double *in = alpha;
    int k = 0;
    for (thx_plan *q = p; q; q = q->next) {
        double *out = q->next ? bufs[(k++) & 1] : beta;
        execute_stage(q, off, deg, in, out, degree, batch, ld, s, sc);
        in = out;
    }
}

// ---- layouts in the static scratch (thx_execute_noalloc) ----
constexpr int64_t SC_ALIGN = 256;
inline int64_t sc_round(int64_t b) { return (b + SC_ALIGN - 1) / SC_ALIGN * SC_ALIGN; }

// Carve one stage's workspace (and its single-precision tail's) from `region`
// with slot chunks of at most `chunk`; returns the bytes used (ws written when
// `out` is set).
int64_t carve_stage(const thx_plan *p, int64_t batch, int64_t chunk, char *region, Ws *w, Ws *wt)
{
    int64_t used = 0;
    auto take = [&](int64_t bytes) -> char * {
        char *q = region ? region + used : nullptr;
        used += sc_round(std::max<int64_t>(bytes, 1));
        return q;
    };
    Ws a, b;
    if (p->path == 4) {
        a.sfx_tot = (double *)take(8 * suffix_tot_doubles(p->kd, p->N, batch));
    } else if (p->path == 1 || p->path == 2) {
        auto one = [&](const thx_plan *q, Ws &x) {
            const int64_t es = (int64_t)q->esize();
            x.U_slots = q->path == 2 ? std::max<int64_t>(1, std::min<int64_t>(chunk, std::max(q->S, 1))) : 0;
            x.X = take(es * batch * q->ncs);
            x.Wp = take(es * groups_for(q, batch, std::max<int64_t>(x.U_slots, 1)) * batch * q->ncs);
            if (q->path == 2) x.U = take(es * q->L * batch * x.U_slots);
        };
        one(p, a);
        a.row0 = (double *)take(8 * batch);
        if (p->row0_direct) a.row0_part = (double *)take(8 * batch * ROW0_PMAX);
        if (p->tail_on && p->tail) one(p->tail, b);
    }
    if (w) *w = a;
    if (wt) *wt = b;
    return used;
}

// Largest slot chunk whose layout fits `bytes`; 0 when none does.
int64_t fit_chunk(const thx_plan *p, int64_t batch, int64_t bytes)
{
    const int64_t smax = std::max<int64_t>(1, std::max(p->S, p->tail ? p->tail->S : 0));
    for (int64_t c = smax; c >= 1; --c)
        if (carve_stage(p, batch, c, nullptr, nullptr, nullptr) <= bytes) return c;
    return 0;
}

void execute_stage(thx_plan *p, const int64_t *off, const int64_t *deg, const double *alpha, double *beta,
                   int64_t degree, int64_t batch, int64_t ld, hipStream_t s, const Scratch *sc)
{
    Ws w, wt;
    if (sc) {
        carve_stage(p, batch, fit_chunk(p, batch, sc->region_bytes), sc->region, &w, &wt);
    } else if (p->path != 0 && degree >= 2) {
        ensure_workspace(p, batch);
        w = own_ws(p);
        if (p->tail) wt = own_ws(p->tail);
    }
    if (p->path == 4 && degree >= 2) {
        PhaseTimer t(p, THX_PHASE_SCAN, s);
        launch_suffix(p->kd, off, deg, alpha, ld, beta, degree, batch, p->tsym, p->hk, w.sfx_tot, s);
        launch_check();
        return;
    }
    if (p->path == 0 || degree < 2) {
        PhaseTimer t(p, THX_PHASE_DIRECT, s);
        launch_direct(p->kd, off, deg, alpha, ld, beta, degree, batch, p->tsym, p->hk, s);
        launch_check();
        return;
    }
    if (p->prec == THX_FP64) execute_fft<double>(p, w, wt, off, deg, alpha, beta, degree, batch, ld, s);
    else execute_fft<float>(p, w, wt, off, deg, alpha, beta, degree, batch, ld, s);
}

// plans whose launches have no per-vector grid limit: the dense product, and a
// single unit step on short vectors (one wave per vector)
bool unlimited_batch(const thx_plan *p, int64_t degree)
{
    return p->dense || (p->path == 4 && !p->next && suffix_small(p->kd, degree));
}

thx_status do_execute(const thx_plan *cp, const double *alpha, double *beta, int64_t degree, int64_t batch,
                      int64_t ld, hipStream_t s)
{
    thx_plan *p = const_cast<thx_plan *>(cp);
    if (!p || degree < 0 || degree > p->N || batch < 0 || ld < degree + 1) return THX_INVALID_ARGUMENT;
    if (batch == 0) return THX_OK;
    if (!alpha || !beta) return THX_INVALID_ARGUMENT;
    if (batch > 65535 && !unlimited_batch(p, degree)) return THX_INVALID_ARGUMENT; // grid.y limit of the launches
    try {
        execute_core(p, nullptr, nullptr, alpha, beta, degree, batch, ld, s, batch * ld);
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        return THX_OUT_OF_MEMORY;
    }
    return THX_OK;
}

// Execution with every workspace buffer in the static scratch: intermediates
// between stages first, then one region the stages use in turn.  Allocates
// nothing and records no events.
thx_status do_execute_noalloc(const thx_plan *cp, const double *alpha, double *beta, int64_t degree,
                              int64_t batch, int64_t ld, hipStream_t s)
{
    thx_plan *p = const_cast<thx_plan *>(cp);
    if (!p || degree < 0 || degree > p->N || batch < 0 || ld < degree + 1) return THX_INVALID_ARGUMENT;
    if (batch == 0) return THX_OK;
    if (!alpha || !beta) return THX_INVALID_ARGUMENT;
    if (batch > 65535 && !unlimited_batch(p, degree)) return THX_INVALID_ARGUMENT;
    hipError_t he = hipSuccess;
    char *base = (char *)scratch_device_ptr(&he);
    if (!base) {
        g_last_hip_error = (int)he;
        return THX_HIP_ERROR;
    }
    Scratch sc;
    sc.base = base;
    sc.bytes = SCRATCH_BYTES;
    int64_t used = 0;
    if (p->next && !p->dense) {
        if (batch > (SCRATCH_BYTES / 8) / ld) return THX_WORKSPACE_TOO_LARGE;
        const int64_t tb = sc_round(8 * batch * ld);
        int stages = 0;
        for (const thx_plan *q = p; q; q = q->next) ++stages;
        sc.tmp = (double *)(base + used);
        used += tb;
        if (stages >= 3) {
            sc.tmp2 = (double *)(base + used);
            used += tb;
        }
        if (used > SCRATCH_BYTES) return THX_WORKSPACE_TOO_LARGE;
    }
    sc.region = base + used;
    sc.region_bytes = SCRATCH_BYTES - used;
    if (!p->dense && degree >= 2)
        for (const thx_plan *q = p; q; q = q->next)
            if (q->path != 0 && fit_chunk(q, batch, sc.region_bytes) == 0) return THX_WORKSPACE_TOO_LARGE;
    g_no_timing = true;
    thx_status st = THX_OK;
    try {
        execute_core(p, nullptr, nullptr, alpha, beta, degree, batch, ld, s, batch * ld, &sc);
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        st = THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        st = THX_OUT_OF_MEMORY;
    }
    g_no_timing = false;
    return st;
}

// Variable-length execution: members at device offsets, degrees derived on the
// device (no host synchronisation), then the same launches as a batch bucket.
thx_status do_execute_varlen(const thx_plan *cp, const double *alpha, double *beta, const int64_t *d_off,
                             int64_t count, int64_t total, int64_t *d_skipped, hipStream_t s)
{
    thx_plan *p = const_cast<thx_plan *>(cp);
    if (!p || count < 0 || total < 0 || (count > 0 && !d_off)) return THX_INVALID_ARGUMENT;
    if (count == 0) return THX_OK;
    if (!alpha || !beta) return THX_INVALID_ARGUMENT;
    if (count > 65535 && !unlimited_batch(p, p->N)) return THX_INVALID_ARGUMENT; // grid.y limit
    try {
        if (count > p->vl_count) {
            dfree(p->vl_off);
            dfree(p->vl_deg);
            p->vl_off = p->vl_deg = nullptr;
            p->vl_count = 0;
            p->vl_off = dalloc<int64_t>(count);
            p->vl_deg = dalloc<int64_t>(count);
            p->vl_count = count;
        }
        launch_varlen(d_off, count, total, p->N, p->vl_off, p->vl_deg, d_skipped, s);
        launch_check();
        execute_core(p, p->vl_off, p->vl_deg, alpha, beta, p->N, count, 0, s, std::max<int64_t>(total, 1));
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        return THX_OUT_OF_MEMORY;
    }
    return THX_OK;
}

// ---- autotuning: launch shapes, row length, dense vs FFT ------------------------
// Candidates are timed with HIP events on zero-filled inputs of the expected
// batch (values do not change the work), median of three after one warm-up.
template <typename F>
float time_launches(F &&run, hipStream_t s)
{
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0));
    hip_check(hipEventCreate(&e1));
    float t[3];
    try {
        run();
        for (float &x : t) {
            hip_check(hipEventRecord(e0, s));
            run();
            hip_check(hipEventRecord(e1, s));
            hip_check(hipEventSynchronize(e1));
            hip_check(hipEventElapsedTime(&x, e0, e1));
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    hip_check(hipEventDestroy(e0));
    hip_check(hipEventDestroy(e1));
    std::sort(t, t + 3);
    return t[1];
}

// rebuild the three-pass tables (row length `row`) from a fresh double spectrum
void configure_rows(thx_plan *p, int64_t row, hipStream_t s)
{
    const bool f64 = p->prec == THX_FP64;
    const MultiPassGeom g = f64 ? multipass_geom<double>(p->L, row) : multipass_geom<float>(p->L, row);
    if (g.L1 == p->geom.L1) return;
    double *spec = symbol_spectrum64(p, s);
    dfree(p->twL1);
    dfree(p->twL2);
    dfree(p->twA);
    dfree(p->that);
    for (double *&q : p->tw64_keep) {
        dfree(q);
        q = nullptr;
    }
    p->twL1 = p->twL2 = p->twA = p->that = nullptr;
    p->geom = g;
    p->twL1 = make_twiddles(p, g.L1, g.L1, s, 0);
    p->twL2 = make_twiddles(p, g.L2, g.L2, s, 1);
    p->twA = make_twiddles(p, p->L, g.L1, s, 2);
    p->that = dalloc<char>((int64_t)p->esize() * p->L);
    if (f64) launch_reorder<double>(spec, p->that, p->L, g.L1, g.L2, 2, s);
    else launch_reorder<float>(spec, p->that, p->L, g.L1, g.L2, 2, s);
    launch_check();
    hip_check(hipStreamSynchronize(s));
    dfree(spec);
}

void tune_stage(thx_plan *p, const double *alpha, double *beta, int64_t batch, hipStream_t s)
{
    auto run = [&] { execute_stage(p, nullptr, nullptr, alpha, beta, p->N, batch, p->N + 1, s); };
    if (p->path == 1) {
        int best = p->lds_blocks, best_r = p->lds_radix;
        float tb = 1e30f;
        for (int radix : {8, 16}) {
            p->lds_radix = radix;
            for (int lb : {256, 512, 1024, 2048}) {
                p->lds_blocks = lb;
                const float t = time_launches(run, s);
                if (t < tb) tb = t, best = lb, best_r = radix;
            }
        }
        p->lds_blocks = best;
        p->lds_radix = best_r;
    } else if (p->path == 2) {
        const bool f64 = p->prec == THX_FP64;
        const int64_t rows[3] = {f64 ? mp_row_short<double>() : mp_row_short<float>(),
                                 f64 ? mp_row_long<double>() : mp_row_long<float>(),
                                 f64 ? mp_row_xl<double>() : mp_row_xl<float>()};
        int64_t best_row = p->geom.L1;
        int best_p3 = p->p3_blocks, best_p1 = 0;
        float tb = 1e30f;
        bool best_fuse = false;
        for (int64_t row : rows) {
            if (row <= 0 || p->L / row < 2 || p->L / row > 1024) continue;
            configure_rows(p, row, s);
            if (p->geom.L1 != row) continue;
            p->p1_blocks = 0;
            float trow = 1e30f;
            int row_p3 = p->p3_blocks;
            bool row_fuse = false;
            for (int fuse = 0; fuse < (p->geom.L2 <= 4 ? 2 : 1); ++fuse) {
                p->fuse_p1 = fuse != 0;
                for (int p3 : {512, 1024, 2048}) {
                    p->p3_blocks = p3;
                    const float t = time_launches(run, s);
                    if (t < trow) trow = t, row_p3 = p3, row_fuse = p->fuse_p1;
                }
            }
            if (trow < tb) tb = trow, best_row = row, best_p3 = row_p3, best_fuse = row_fuse, best_p1 = 0;
            // then, for this row length, the separate forward column pass with
            // several slots per workgroup (when that still leaves enough
            // workgroups): its tiles differ per row length, so it is timed
            // with each
            if (!row_fuse) {
                p->p3_blocks = row_p3;
                p->fuse_p1 = false;
                for (int p1 : {8192, 2048}) {
                    p->p1_blocks = p1;
                    const float t = time_launches(run, s);
                    if (t < tb) tb = t, best_row = row, best_p3 = row_p3, best_fuse = false, best_p1 = p1;
                }
            }
        }
        configure_rows(p, best_row, s);
        p->p3_blocks = best_p3;
        p->fuse_p1 = best_fuse;
        p->p1_blocks = best_p1;
        // single-precision tail on (with its inverse-pass workgroups) or off
        // (off: those slots in double precision)
        if (p->tail) {
            const int s64 = p->S_full - p->tail->S;
            p->tail_on = false;
            p->S = p->S_full;
            float tb_tail = time_launches(run, s);
            bool best_on = false;
            int best_tp3 = p->tail->p3_blocks;
            p->tail_on = true;
            p->S = s64;
            for (int p3 : {512, 1024, 2048}) {
                p->tail->p3_blocks = p3;
                const float t = time_launches(run, s);
                if (t < tb_tail) tb_tail = t, best_on = true, best_tp3 = p3;
            }
            p->tail->p3_blocks = best_tp3;
            p->tail_on = best_on;
            p->S = best_on ? s64 : p->S_full;
        }
    }
}

thx_status autotune(thx_plan *p, int64_t batch, hipStream_t s)
{
    if (!p || batch < 1) return THX_INVALID_ARGUMENT;
    const int64_t n1 = p->N + 1;
    const int64_t fb = std::min<int64_t>(batch, 65535); // the FFT launches' grid limit
    double *a = nullptr, *b = nullptr;
    try {
        a = dalloc<double>(batch * n1);
        b = dalloc<double>(batch * n1);
        launch_zero(a, batch * n1 * (int64_t)sizeof(double), s);
        // bring the clocks up before the first candidate is timed: a GPU coming out
        // of idle runs the first few milliseconds of work slower, which favoured the
        // candidates timed last
        for (thx_plan *q = p; q; q = q->next) {
            if (q->path == 0 || p->N < 2) continue;
            ensure_workspace(q, fb);
            const auto t0 = std::chrono::steady_clock::now();
            for (int it = 0; it < 256; ++it) {
                execute_stage(q, nullptr, nullptr, a, b, q->N, fb, q->N + 1, s);
                hip_check(hipStreamSynchronize(s));
                if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(15)) break;
            }
            break;
        }
        for (thx_plan *q = p; q; q = q->next) {
            if (q->path == 0 || p->N < 2) continue;
            ensure_workspace(q, fb);
            tune_stage(q, a, b, fb, s);
        }
        // dense product vs the stages' own paths, for the whole conversion
        bool fft_capable = false;
        for (const thx_plan *q = p; q; q = q->next) fft_capable |= q->path != 0;
        if (fft_capable && !(p->flags & (THX_FLAG_FORCE_FFT | THX_FLAG_NO_DENSE)) && n1 <= DENSE_TUNE_MAX) {
            double *keep = p->dense;
            uint16_t *keep_bf = p->dense_bf;
            p->dense = nullptr;
            p->dense_bf = nullptr;
            const float t_fft = time_launches([&] { execute_core(p, nullptr, nullptr, a, b, p->N, fb, n1, s, fb * n1); }, s);
            if (keep) {
                p->dense = keep;
                p->dense_bf = keep_bf;
            } else {
                build_dense(p, s);
            }
            const float t_dense = time_launches([&] { execute_core(p, nullptr, nullptr, a, b, p->N, fb, n1, s, fb * n1); }, s);
            if (t_fft < t_dense) drop_dense(p);
        }
        hip_check(hipStreamSynchronize(s));
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        dfree(a);
        dfree(b);
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        dfree(a);
        dfree(b);
        return THX_OUT_OF_MEMORY;
    }
    dfree(a);
    dfree(b);
    return THX_OK;
}

// ---- plan cache for the one-shot calls ----
// One plan per (kind, parameters, degree, tol, precision, device).  Calls with
// the same key share the plan's workspace, so they are serialised: the host side
// holds the entry's mutex while it launches, and the launches wait (on the
// device) for the previous call's work through the entry's event, whatever
// stream that call used.  Before the workspace may be reallocated for a larger
// batch, the previous call's work is waited for on the host.
using Key = std::tuple<int, double, double, double, double, int64_t, double, int, int>;
struct CacheEntry {
    thx_plan *p = nullptr;
    std::mutex mu;
    hipEvent_t done = nullptr; // recorded after each call's launches
    ~CacheEntry()
    {
        if (done) (void)hipEventDestroy(done);
        delete p;
    }
};
std::mutex g_cache_mu;
std::map<Key, std::unique_ptr<CacheEntry>> g_cache;

// true when executing `batch` vectors of `elems` coefficients in all may grow
// (free and reallocate) a workspace of the plan
bool may_reallocate(const thx_plan *p, int64_t batch, int64_t elems)
{
    if (p->dense) return false;
    if (p->next && p->tmp_elems < elems) return true;
    for (const thx_plan *q = p; q; q = q->next)
        if (q->path != 0 && q->ws_batch < batch) return true;
    return false;
}

thx_status cached_convert(thx_kind kind, const double *params, int np, const double *alpha, double *beta,
                          int64_t N, int64_t batch, double tol, thx_precision prec, hipStream_t s)
{
    if (N < 0) return THX_INVALID_ARGUMENT;
    int dev = 0;
    (void)hipGetDevice(&dev);
    double kp[4] = {0, 0, 0, 0};
    for (int i = 0; i < np && i < 4; ++i) kp[i] = params[i];
    const Key k{(int)kind, kp[0], kp[1], kp[2], kp[3], N, tol, (int)prec, dev};
    CacheEntry *e = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(k);
        if (it != g_cache.end()) e = it->second.get();
    }
    if (!e) {
        thx_plan *p = nullptr;
        thx_status st = create_plan(&p, kind, params, np, N, tol, prec, 0, s);
        if (st != THX_OK && st != THX_TOL_NOT_REACHED) return st;
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(k);
        if (it != g_cache.end()) {
            delete p;
        } else {
            std::unique_ptr<CacheEntry> ne(new (std::nothrow) CacheEntry());
            if (!ne) {
                delete p;
                return THX_OUT_OF_MEMORY;
            }
            ne->p = p;
            hipError_t he = hipEventCreateWithFlags(&ne->done, hipEventDisableTiming);
            if (he != hipSuccess) {
                g_last_hip_error = (int)he;
                return THX_HIP_ERROR;
            }
            it = g_cache.emplace(k, std::move(ne)).first;
        }
        e = it->second.get();
    }
    std::lock_guard<std::mutex> lk(e->mu);
    hipError_t he = hipStreamWaitEvent(s, e->done, 0);
    if (he == hipSuccess && may_reallocate(e->p, batch, batch * (N + 1))) he = hipEventSynchronize(e->done);
    if (he != hipSuccess) {
        g_last_hip_error = (int)he;
        return THX_HIP_ERROR;
    }
    const thx_status st = do_execute(e->p, alpha, beta, N, batch, N + 1, s);
    he = hipEventRecord(e->done, s);
    if (st == THX_OK && he != hipSuccess) {
        g_last_hip_error = (int)he;
        return THX_HIP_ERROR;
    }
    return st;
}

// ---- mixed-degree batches (CSR layout), one plan per FFT-length bucket ----
} // namespace

struct thx_batch {
    struct Bucket {
        thx_plan *plan = nullptr;
        int64_t members = 0, Nmax = 0, L = 0;
        int64_t *d_off = nullptr, *d_deg = nullptr;
        int lane = 0; // 0: the caller's (or capture) stream, 1: side_stream
    };
    int64_t count = 0, total = 0;
    std::vector<Bucket> buckets;
    hipStream_t cap_stream = nullptr;
    // Buckets read and write disjoint coefficients, so the FFT buckets run in two
    // lanes: one bucket's launch ramps and short single-workgroup transforms
    // overlap another's HBM-bound passes (the dense product and the unit steps stay
    // in the first lane: overlapped with each other they measured slower, e.g.
    // 0.183 against 0.170 ms for the unit steps of 65536 vectors of degree 255
    // beside 64 of degree 2^18).  The
    // side lane forks from and joins the calling stream through events, also under
    // capture (the graph then has two branches).
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *g_alpha = nullptr;
    double *g_beta = nullptr;
    ~thx_batch()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (side_stream) (void)hipStreamDestroy(side_stream);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        for (auto &b : buckets) {
            delete b.plan;
            dfree(b.d_off);
            dfree(b.d_deg);
        }
    }
};

namespace {

constexpr int64_t MAX_BUCKET_MEMBERS = 65535; // grid.y limit of the per-vector launches

// Rough cost of one execution of a bucket, to balance the two lanes: FFT work
// ~ members L K, the dense product ~ members (N+1)^2 on the matrix cores, the
// direct evaluation ~ members (N+1)^2 on the vector units, a unit step ~ members
// (N+1).
double bucket_cost(const thx_batch::Bucket &bk)
{
    const double n1 = (double)bk.Nmax + 1, m = (double)bk.members;
    const thx_plan *p = bk.plan;
    if (p->dense) return m * n1 * n1 / 64;
    if (p->path == 0) return m * n1 * n1 / 8;
    if (p->path == 4) return 3 * m * n1;
    return m * (double)p->L * std::max(1, std::max(p->S, p->S_full));
}

bool bucket_is_fft(const thx_batch::Bucket &bk)
{
    return !bk.plan->dense && (bk.plan->path == 1 || bk.plan->path == 2);
}

// Longest-first assignment of the FFT buckets to the lane with less work so far
// (the others stay in lane 0, counted there); the launch order within a lane
// stays the bucket order.
void assign_lanes(thx_batch *b)
{
    std::vector<size_t> order;
    double load[2] = {0, 0};
    for (size_t i = 0; i < b->buckets.size(); ++i) {
        if (bucket_is_fft(b->buckets[i])) order.push_back(i);
        else load[0] += bucket_cost(b->buckets[i]);
    }
    std::sort(order.begin(), order.end(),
              [&](size_t x, size_t y) { return bucket_cost(b->buckets[x]) > bucket_cost(b->buckets[y]); });
    for (size_t i : order) {
        const int lane = load[1] < load[0] ? 1 : 0;
        b->buckets[i].lane = lane;
        load[lane] += bucket_cost(b->buckets[i]);
    }
}

thx_status batch_create(thx_batch **out, thx_kind kind, const double *params, int nparams, const int64_t *degrees,
                        int64_t count, double tol, thx_precision prec, uint32_t flags, hipStream_t s)
{
    if (!out) return THX_INVALID_ARGUMENT;
    *out = nullptr;
    if (count < 0 || (count > 0 && !degrees)) return THX_INVALID_ARGUMENT;
    for (int64_t i = 0; i < count; ++i)
        if (degrees[i] < 0) return THX_INVALID_ARGUMENT;
    double pv[4] = {0, 0, 0, 0};
    thx_status vs = validate_kind(kind, params, nparams, pv);
    if (vs != THX_OK) return vs;
    const bool parity = (kind == THX_LEG2CHEB || kind == THX_CHEB2LEG || kind == THX_ULTRA2ULTRA);
    thx_batch *b = new (std::nothrow) thx_batch();
    if (!b) return THX_OUT_OF_MEMORY;
    b->count = count;
    // bucket key: 0 for the direct evaluation, else the FFT length
    std::map<int64_t, std::vector<int64_t>> groups;
    std::vector<int64_t> off(count);
    int64_t acc = 0;
    for (int64_t i = 0; i < count; ++i) {
        off[i] = acc;
        acc += degrees[i] + 1;
        const int64_t N = degrees[i];
        const bool direct = (flags & THX_FLAG_FORCE_DIRECT) ||
                            (!(flags & THX_FLAG_FORCE_FFT) && N <= direct_crossover()) || N < 2;
        const int64_t nc = parity ? N / 2 + 1 : N + 1;
        groups[direct ? 0 : fft_length_for(nc, prec)].push_back(i);
    }
    b->total = acc;
    thx_status result = THX_OK;
    try {
        for (auto &kv : groups) {
            const std::vector<int64_t> &idx = kv.second;
            // the dense product has no per-vector grid limit: one bucket
            int64_t gmax = 0;
            for (int64_t i : idx) gmax = std::max(gmax, degrees[i]);
            // with autotuning, an FFT bucket keeps its FFT plan and may still pick the dense product
            const uint32_t f = (kv.first == 0 ? FLAG_SHORT
                                              : ((flags & THX_FLAG_AUTOTUNE) ? 0u : THX_FLAG_FORCE_FFT)) |
                               (flags & THX_FLAG_NO_DENSE);
            // more members than one grid dimension holds: one bucket if the plan for the
            // whole group has no per-vector grid limit, else chunks of MAX_BUCKET_MEMBERS
            thx_plan *whole = nullptr;
            size_t chunk = (size_t)MAX_BUCKET_MEMBERS;
            if (idx.size() > chunk) {
                thx_status st = create_plan(&whole, kind, params, nparams, gmax, tol, prec, f, s);
                if (st != THX_OK && st != THX_TOL_NOT_REACHED) {
                    delete b;
                    return st;
                }
                if (unlimited_batch(whole, gmax)) {
                    chunk = idx.size();
                } else {
                    delete whole;
                    whole = nullptr;
                }
            }
            for (size_t c0 = 0; c0 < idx.size(); c0 += chunk) {
                const size_t c1 = std::min(idx.size(), c0 + chunk);
                thx_batch::Bucket bk;
                std::vector<int64_t> ho, hd;
                for (size_t m = c0; m < c1; ++m) {
                    ho.push_back(off[idx[m]]);
                    hd.push_back(degrees[idx[m]]);
                    bk.Nmax = std::max(bk.Nmax, degrees[idx[m]]);
                }
                bk.members = (int64_t)ho.size();
                thx_status st = THX_OK;
                if (whole) {
                    bk.plan = whole; // the group's plan, made above at its largest degree
                    whole = nullptr;
                } else {
                    st = create_plan(&bk.plan, kind, params, nparams, bk.Nmax, tol, prec, f, s);
                }
                if (st == THX_TOL_NOT_REACHED) result = st;
                else if (st != THX_OK) {
                    delete b;
                    return st;
                }
                if (flags & THX_FLAG_AUTOTUNE) {
                    thx_status ts = autotune(bk.plan, bk.members, s);
                    if (ts != THX_OK) {
                        delete bk.plan;
                        delete b;
                        return ts;
                    }
                }
                if (!unlimited_batch(bk.plan, bk.Nmax) && bk.members > MAX_BUCKET_MEMBERS) {
                    delete bk.plan;
                    delete b;
                    return THX_UNSUPPORTED;
                }
                bk.L = (bk.plan->path == 0 || bk.plan->dense) ? 0 : bk.plan->L;
                bk.d_off = dalloc<int64_t>(bk.members);
                bk.d_deg = dalloc<int64_t>(bk.members);
                hip_check(hipMemcpyAsync(bk.d_off, ho.data(), sizeof(int64_t) * ho.size(), hipMemcpyHostToDevice, s));
                hip_check(hipMemcpyAsync(bk.d_deg, hd.data(), sizeof(int64_t) * hd.size(), hipMemcpyHostToDevice, s));
                if (!bk.plan->dense) {
                    for (thx_plan *q = bk.plan; q; q = q->next)
                        if (q->path != 0) ensure_workspace(q, bk.members);
                    if (bk.plan->next) ensure_tmp(bk.plan, acc);
                }
                b->buckets.push_back(bk);
                hip_check(hipStreamSynchronize(s));
            }
        }
        hip_check(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        int fft_buckets = 0;
        for (const auto &bk : b->buckets) fft_buckets += bucket_is_fft(bk) ? 1 : 0;
        if (fft_buckets > 1) {
            hip_check(hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking));
            hip_check(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
            hip_check(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
            assign_lanes(b);
        }
    } catch (const HipFail &e) {
        g_last_hip_error = (int)e.e;
        delete b;
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        delete b;
        return THX_OUT_OF_MEMORY;
    }
    *out = b;
    return result;
}

void batch_launch(thx_batch *b, const double *alpha, double *beta, hipStream_t s)
{
    if (!b->side_stream) {
        for (auto &bk : b->buckets)
            execute_core(bk.plan, bk.d_off, bk.d_deg, alpha, beta, bk.Nmax, bk.members, 0, s, b->total);
        return;
    }
    hip_check(hipEventRecord(b->ev_fork, s));
    hip_check(hipStreamWaitEvent(b->side_stream, b->ev_fork, 0));
    for (auto &bk : b->buckets)
        execute_core(bk.plan, bk.d_off, bk.d_deg, alpha, beta, bk.Nmax, bk.members, 0,
                     bk.lane ? b->side_stream : s, b->total);
    hip_check(hipEventRecord(b->ev_join, b->side_stream));
    hip_check(hipStreamWaitEvent(s, b->ev_join, 0));
}

thx_status batch_execute(thx_batch *b, const double *alpha, double *beta, int use_graph, hipStream_t s)
{
    if (!b) return THX_INVALID_ARGUMENT;
    if (b->count == 0) return THX_OK;
    if (!alpha || !beta) return THX_INVALID_ARGUMENT;
    try {
        if (!use_graph) {
            batch_launch(b, alpha, beta, s);
            return THX_OK;
        }
        if (!b->gexec || b->g_alpha != alpha || b->g_beta != beta) {
            if (b->gexec) {
                hip_check(hipGraphExecDestroy(b->gexec));
                b->gexec = nullptr;
            }
            // capture on the batch's own stream, replay on the caller's
            hip_check(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            try {
                batch_launch(b, alpha, beta, b->cap_stream);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(b->cap_stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            hipGraph_t g = nullptr;
            hip_check(hipStreamEndCapture(b->cap_stream, &g));
            hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            hip_check(e);
            b->g_alpha = alpha;
            b->g_beta = beta;
        }
        hip_check(hipGraphLaunch(b->gexec, s));
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        return THX_HIP_ERROR;
    } catch (const std::bad_alloc &) {
        return THX_OUT_OF_MEMORY;
    }
    return THX_OK;
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

constexpr uint32_t PUBLIC_FLAGS = THX_FLAG_FORCE_DIRECT | THX_FLAG_FORCE_FFT | THX_FLAG_NO_DENSE | THX_FLAG_AUTOTUNE;

thx_status thx_plan_create(thx_plan **out, thx_kind kind, const double *params, int nparams, int64_t degree,
                           double tol, thx_precision prec, uint32_t flags, hipStream_t stream)
{
    return create_plan(out, kind, params, nparams, degree, tol, prec, flags & PUBLIC_FLAGS, stream);
}

thx_status thx_execute(const thx_plan *plan, const double *alpha, double *beta, int64_t degree, int64_t batch,
                       int64_t ld, hipStream_t stream)
{
    return do_execute(plan, alpha, beta, degree, batch, ld, stream);
}

thx_status thx_plan_destroy(thx_plan *plan)
{
    delete plan;
    return THX_OK;
}

int32_t thx_plan_rank(const thx_plan *p)
{
    if (!p) return -1;
    int32_t r = 0;
    for (const thx_plan *q = p; q; q = q->next) r = std::max<int32_t>(r, q->path == 0 ? 0 : std::max(q->S, q->S_full));
    return r;
}
int32_t thx_plan_tail_slots(const thx_plan *p)
{
    if (!p) return -1;
    int32_t r = 0;
    for (const thx_plan *q = p; q; q = q->next)
        if (q->tail && q->tail_on && !p->dense) r += q->tail->S;
    return r;
}
int32_t thx_plan_rank_part(const thx_plan *p, int part)
{
    if (!p || part < 0 || part >= p->parts || p->path == 0) return -1;
    return p->K[part];
}
int64_t thx_plan_fft_length(const thx_plan *p)
{
    if (!p) return -1;
    int64_t L = 0;
    if (p->dense) return 0;
    for (const thx_plan *q = p; q; q = q->next) L = std::max<int64_t>(L, (q->path == 1 || q->path == 2) ? q->L : 0);
    return L;
}
int32_t thx_plan_path(const thx_plan *p) { return p ? (p->dense ? 3 : p->path) : -1; }
thx_status thx_plan_launch_shape(const thx_plan *p, int32_t *lds_blocks, int32_t *p3_blocks)
{
    if (!p) return THX_INVALID_ARGUMENT;
    if (lds_blocks) *lds_blocks = p->lds_blocks;
    if (p3_blocks) *p3_blocks = p->p3_blocks;
    return THX_OK;
}
int32_t thx_plan_lds_radix(const thx_plan *p) { return p ? p->lds_radix : -1; }
int32_t thx_plan_p1_blocks(const thx_plan *p) { return p ? p->p1_blocks : -1; }
int32_t thx_plan_fused_columns(const thx_plan *p)
{
    if (!p) return -1;
    return (p->path == 2 && !p->dense && p->fuse_p1 && p->geom.L2 <= 4) ? 1 : 0;
}

int32_t thx_plan_partial_groups(const thx_plan *p, int64_t batch)
{
    if (!p || batch < 1 || p->dense || p->S <= 0) return 0;
    if (p->path == 1) {
        const int64_t Gt = std::min<int64_t>(p->S, std::max<int64_t>(1, (p->lds_blocks + batch - 1) / batch));
        const int64_t spg = (p->S + Gt - 1) / Gt;
        return (int32_t)((p->S + spg - 1) / spg);
    }
    if (p->path != 2) return 0;
    const int64_t tiles = p->geom.L1 / p->geom.TC;
    int64_t G = 0;
    for (int64_t s0 = 0; s0 < p->S; s0 += std::max<int64_t>(1, p->U_slots ? p->U_slots : p->S)) {
        const int64_t ns = std::min<int64_t>(p->U_slots ? p->U_slots : p->S, p->S - s0);
        int64_t Gc = std::min<int64_t>(ns, std::max<int64_t>(1, (p->p3_blocks + tiles * batch - 1) / (tiles * batch)));
        const int64_t spg = (ns + Gc - 1) / Gc;
        G += (ns + spg - 1) / spg;
    }
    return (int32_t)G;
}

thx_status thx_plan_fft_geometry(const thx_plan *p, int64_t *rows, int64_t *cols, int64_t *tile_cols)
{
    if (!p || p->path != 2 || p->dense) return THX_INVALID_ARGUMENT;
    if (rows) *rows = p->geom.L1;
    if (cols) *cols = p->geom.L2;
    if (tile_cols) *tile_cols = p->geom.TC;
    return THX_OK;
}
double thx_plan_achieved_tol(const thx_plan *p, int part)
{
    if (!p || part < 0 || part >= p->parts || p->path == 0 || p->path == 4) return -1.0;
    return p->dfinal[part] * p->escale[part];
}

thx_status thx_plan_factors(const thx_plan *p, int part, double *ell, int32_t *pivots, int64_t *n_out,
                            hipStream_t stream)
{
    if (!p || part < 0 || part >= p->parts || p->path == 0) return THX_INVALID_ARGUMENT;
    const int64_t n = p->npart[part];
    if (n_out) *n_out = n;
    if (pivots)
        for (int r = 0; r < p->K[part]; ++r) pivots[r] = p->pivots[part][r];
    if (!ell) return THX_OK;
    try {
        std::vector<double> h(2 * (size_t)p->slots_alloc * p->ncs);
        hip_check(hipMemcpyAsync(h.data(), p->ell64, sizeof(double) * h.size(), hipMemcpyDeviceToHost, stream));
        hip_check(hipStreamSynchronize(stream));
        for (int r = 0; r < p->K[part]; ++r)
            for (int64_t i = 0; i < n; ++i) {
                const int64_t idx = p->parts == 2 ? 2 * ((int64_t)r * p->ncs + i) + part
                                                  : 2 * ((int64_t)(r >> 1) * p->ncs + i) + (r & 1);
                ell[(int64_t)r * n + i] = h[idx];
            }
    } catch (const HipFail &f) {
        g_last_hip_error = (int)f.e;
        return THX_HIP_ERROR;
    }
    return THX_OK;
}

thx_status thx_leg2cheb(const double *alpha, double *beta, int64_t N, int64_t batch, double tol,
                        thx_precision prec, hipStream_t stream)
{
    return cached_convert(THX_LEG2CHEB, nullptr, 0, alpha, beta, N, batch, tol, prec, stream);
}
thx_status thx_cheb2leg(const double *alpha, double *beta, int64_t N, int64_t batch, double tol,
                        thx_precision prec, hipStream_t stream)
{
    return cached_convert(THX_CHEB2LEG, nullptr, 0, alpha, beta, N, batch, tol, prec, stream);
}
thx_status thx_ultra2ultra(const double *alpha, double *beta, int64_t N, int64_t batch, double lambda1,
                           double lambda2, double tol, thx_precision prec, hipStream_t stream)
{
    const double p[2] = {lambda1, lambda2};
    return cached_convert(THX_ULTRA2ULTRA, p, 2, alpha, beta, N, batch, tol, prec, stream);
}
thx_status thx_lag2lag(const double *alpha, double *beta, int64_t N, int64_t batch, double alpha1,
                       double alpha2, double tol, thx_precision prec, hipStream_t stream)
{
    const double p[2] = {alpha1, alpha2};
    return cached_convert(THX_LAG2LAG, p, 2, alpha, beta, N, batch, tol, prec, stream);
}

thx_status thx_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto &kv : g_cache) {
        // wait for a call of another thread that is still launching, then for its work
        std::lock_guard<std::mutex> le(kv.second->mu);
        (void)hipEventSynchronize(kv.second->done);
    }
    if (!g_cache.empty()) (void)hipDeviceSynchronize();
    g_cache.clear();
    return THX_OK;
}

thx_status thx_jac2jac(const double *alpha, double *beta, int64_t N, int64_t batch, double a, double b, double g,
                       double d, double tol, thx_precision prec, hipStream_t stream)
{
    const double p[4] = {a, b, g, d};
    return cached_convert(THX_JAC2JAC, p, 4, alpha, beta, N, batch, tol, prec, stream);
}
thx_status thx_jac2cheb(const double *alpha, double *beta, int64_t N, int64_t batch, double a, double b,
                        double tol, thx_precision prec, hipStream_t stream)
{
    const double p[2] = {a, b};
    return cached_convert(THX_JAC2CHEB, p, 2, alpha, beta, N, batch, tol, prec, stream);
}
thx_status thx_cheb2jac(const double *alpha, double *beta, int64_t N, int64_t batch, double g, double d,
                        double tol, thx_precision prec, hipStream_t stream)
{
    const double p[2] = {g, d};
    return cached_convert(THX_CHEB2JAC, p, 2, alpha, beta, N, batch, tol, prec, stream);
}

thx_status thx_execute_noalloc(const thx_plan *plan, const double *alpha, double *beta, int64_t degree,
                               int64_t batch, int64_t ld, hipStream_t stream)
{
    return do_execute_noalloc(plan, alpha, beta, degree, batch, ld, stream);
}

int64_t thx_noalloc_scratch_bytes(void) { return SCRATCH_BYTES; }

thx_status thx_trace_marker(int id, hipStream_t stream)
{
    if (id < 1 || id > 65535) return THX_INVALID_ARGUMENT;
    launch_trace_marker(id, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip_error = (int)e;
        return THX_HIP_ERROR;
    }
    return THX_OK;
}

thx_status thx_execute_varlen(const thx_plan *plan, const double *alpha, double *beta, const int64_t *d_offsets,
                              int64_t count, int64_t total, int64_t *d_skipped, hipStream_t stream)
{
    return do_execute_varlen(plan, alpha, beta, d_offsets, count, total, d_skipped, stream);
}

thx_status thx_lambda_table(double *out, int64_t count, double z0, hipStream_t stream)
{
    if (count < 0 || (count > 0 && !out)) return THX_INVALID_ARGUMENT;
    launch_gamma_ratio(out, count, z0, make_gamma_ratio(0.5, 1.0), 1.0, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip_error = (int)e;
        return THX_HIP_ERROR;
    }
    return THX_OK;
}

thx_status thx_gamma_ratio_table(double *out, int64_t count, double z0, double a, double b, hipStream_t stream)
{
    if (count < 0 || (count > 0 && !out) || !std::isfinite(a) || !std::isfinite(b)) return THX_INVALID_ARGUMENT;
    launch_gamma_ratio(out, count, z0, make_gamma_ratio(a, b), 1.0, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip_error = (int)e;
        return THX_HIP_ERROR;
    }
    return THX_OK;
}

thx_status thx_plan_autotune(thx_plan *plan, int64_t batch, hipStream_t stream)
{
    return autotune(plan, batch, stream);
}

thx_status thx_plan_enable_timing(thx_plan *p, uint32_t phases)
{
    if (!p) return THX_INVALID_ARGUMENT;
    p->timing = phases & ((1u << THX_NPHASES) - 1u);
    return THX_OK;
}

thx_status thx_plan_timings(thx_plan *p, double *ms, int64_t *launches, int reset)
{
    if (!p) return THX_INVALID_ARGUMENT;
    double acc[THX_NPHASES] = {0};
    int64_t cnt[THX_NPHASES] = {0};
    for (const auto &m : p->marks) {
        hipError_t e = hipEventSynchronize(m.b);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, m.a, m.b);
        if (e != hipSuccess) {
            g_last_hip_error = (int)e;
            return THX_HIP_ERROR;
        }
        acc[m.phase] += (double)t;
        cnt[m.phase] += 1;
    }
    for (int i = 0; i < THX_NPHASES; ++i) {
        if (ms) ms[i] = acc[i];
        if (launches) launches[i] = cnt[i];
    }
    if (reset) p->marks.clear();
    return THX_OK;
}

thx_status thx_batch_create(thx_batch **out, thx_kind kind, const double *params, int nparams,
                            const int64_t *degrees, int64_t count, double tol, thx_precision prec,
                            uint32_t flags, hipStream_t stream)
{
    return batch_create(out, kind, params, nparams, degrees, count, tol, prec, flags & PUBLIC_FLAGS, stream);
}

thx_status thx_batch_execute(thx_batch *batch, const double *alpha, double *beta, int use_graph,
                             hipStream_t stream)
{
    return batch_execute(batch, alpha, beta, use_graph, stream);
}

thx_status thx_batch_destroy(thx_batch *batch)
{
    delete batch;
    return THX_OK;
}

int64_t thx_batch_coefficients(const thx_batch *b) { return b ? b->total : -1; }
int32_t thx_batch_buckets(const thx_batch *b) { return b ? (int32_t)b->buckets.size() : -1; }

thx_status thx_batch_bucket_info(const thx_batch *b, int i, int64_t *fft_length, int64_t *members,
                                 int64_t *max_degree, int32_t *path, int32_t *rank)
{
    if (!b || i < 0 || i >= (int)b->buckets.size()) return THX_INVALID_ARGUMENT;
    const auto &bk = b->buckets[i];
    if (fft_length) *fft_length = bk.L;
    if (members) *members = bk.members;
    if (max_degree) *max_degree = bk.Nmax;
    if (path) *path = thx_plan_path(bk.plan);
    if (rank) *rank = thx_plan_rank(bk.plan);
    return THX_OK;
}

const char *thx_status_string(thx_status s)
{
    switch (s) {
    case THX_OK: return "THX_OK";
    case THX_INVALID_ARGUMENT: return "THX_INVALID_ARGUMENT";
    case THX_UNSUPPORTED: return "THX_UNSUPPORTED";
    case THX_TOL_NOT_REACHED: return "THX_TOL_NOT_REACHED";
    case THX_OUT_OF_MEMORY: return "THX_OUT_OF_MEMORY";
    case THX_HIP_ERROR: return "THX_HIP_ERROR";
    case THX_WORKSPACE_TOO_LARGE: return "THX_WORKSPACE_TOO_LARGE";
    }
    return "THX_UNKNOWN";
}

hipError_t thx_last_hip_error(void) { return (hipError_t)g_last_hip_error; }

} // extern "C"
