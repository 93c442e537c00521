// launch.hpp -- host-side launchers of the libthx kernels (kernels.hip) and the
// small POD descriptors they take.  Everything here is internal to libthx.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace thx {

// Asymptotic series of log(Gamma(z+a)/Gamma(z+b)) in w = z + (a+b-1)/2:
//   (a-b) log w + sum_{j>=1} c_j w^{-2j},  c_j = -B_{2j+1}((1+a-b)/2) / (j(2j+1)),
// where B_n is the Bernoulli polynomial (the odd powers of 1/w vanish with this
// shift).  Used for w >= 12; smaller arguments are shifted up with
// Gamma(x+1) = x Gamma(x).
constexpr int GR_TERMS = 10;
struct GammaRatio {
    double a, b, amb;
    double c[GR_TERMS];
    int pow_mode; // -1: w^{-1/2}, +1: w^{1/2}, 0: pow(w, a-b)
};
GammaRatio make_gamma_ratio(double a, double b);

// Diagonal factors D1, D2 of A = D1 (T o H) D2 for the kinds whose diagonals
// have a short closed form (the others pass tables).
struct KindDesc {
    int kind;     // thx_kind
    int parity;   // 1: A_jk = 0 for odd k - j (split into even/odd halves)
    double p[4];  // kind parameters
    const double *d1tab; // optional D1 table (length >= N+1), else closed form
    const double *d2tab; // optional D2 table
    int64_t band;        // >= 0: A_jk = 0 for k - j > band (identity stages); -1: full
};

// The vectors of an execution in place of a packed X: lane a of vector b is
// (D2 alpha) at indices 2a, 2a+1 (parity kinds) or (D2 alpha)_a twice, as the
// pack step would form it; off / deg and ld / N0 as for launch_pack.
struct AlphaIn {
    KindDesc k;
    const int64_t *off, *deg;
    const double *alpha;
    int64_t ld, N0;
};

// Device state of the pivoted Cholesky (two independent parts at most).
// Pivots are chosen and the factorisation stopped on the weighted residual
// diagonal w_i d_i, w_i = |D1_j D2_j| (the diagonal of S H S with
// S = diag(sqrt|D1 D2|)); see k_pchol_amp for the threshold.
constexpr int KMAX = 128;
struct PcholState {
    int K[2];
    int done[2];
    int active[2];
    int cur_p[2];
    double cur_piv[2];    // unweighted residual diagonal at the current pivot
    double dmax0[2];      // largest weighted diagonal w_i H_ii
    double dfinal[2];     // largest weighted residual at termination / dmax0
    double eps[2];        // stopping threshold relative to dmax0
    double escale[2];     // amp Tmax / (2 |t_0|): dfinal in units of the API tolerance
    int piv[2][KMAX];
    double pval[2][KMAX]; // weighted pivot values (w_p d_p when chosen)
    double R[2][KMAX][KMAX]; // R[q][r][i] = normalised column i of part q at pivot p_r
};

// ---- a1: tables --------------------------------------------------------------
void launch_gamma_ratio(double *out, int64_t count, double z0, const GammaRatio &g, double scale,
                        hipStream_t s);
// tw[k] = exp(-2 pi i k / M), k < count
void launch_twiddles(double *tw64, float *tw32, int64_t M, int64_t count, hipStream_t s);
void launch_cast(const double *in, float *out, int64_t count, hipStream_t s);
void launch_set_value(double *p, double v, hipStream_t s);
void launch_case3_origin(double *hk, const double *d1, double *d2, hipStream_t s);
// D1 (which = 1) or D2 (which = 2) of a Jacobi stage (a, b) -> (g, b), see kernels.hip
void launch_jacobi_diag(double *out, int64_t count, int which, double a, double b, double g, int reflect,
                        int cheb, hipStream_t s);

// ---- a2: pivoted Cholesky ------------------------------------------------------
// parts: 2 for parity-split kinds (even/odd, generator h_q(s) = hk[s + q]),
// 1 otherwise (generator hk[s]).  n[q]: part sizes; a0[q]: first index taking
// part (rows below are excluded).  ell: [KMAX slots][nc] complex doubles.
struct PcholArgs {
    const double *hk;
    double *w;        // pivot weights |D1_j D2_j| [parts][nc] (zero outside a part)
    double *d;        // residual diagonals [parts][nc]
    double *ell;      // (double*) of the complex [slot][nc] array
    int64_t nc;
    int64_t n[2];
    int64_t a0[2];
    int parts;
    double tol;
    int kcap;
    PcholState *st;
    double *pv;       // block partial maxima [parts][nblk]
    int *pi;          // block partial argmax [parts][nblk]
    int nblk;
};
// Weights w and, per part, the threshold eps = max(floor, 2 tol |t_0| / (amp Tmax))
// with amp = max_{j <= k} r_j / r_k, r = sqrt|D1 / D2| and Tmax = max |t_m| over
// the first nt symbol entries; then |beta error| <= 2 tol max_j |A_jj| ||alpha||_1
// for the truncation.  Writes st->eps and st->escale.
void launch_pchol_weights(const KindDesc &k, const PcholArgs &a, const double *tsym, int64_t nt, double tol,
                          double floor_rel, hipStream_t s);
void launch_pchol_init(const PcholArgs &a, hipStream_t s);
void launch_pchol_step(const PcholArgs &a, int r, hipStream_t s);

// ---- a3: Toeplitz symbol -------------------------------------------------------
// embed t_m (m < nt) as the first column of the circulant of length L that
// realises the upper-triangular Toeplitz product as a circular correlation.
void launch_symbol_embed(const double *t, int64_t nt, double *emb /*complex L*/, int64_t L,
                         hipStream_t s);

// reorder a double spectrum into working precision T: mode 0 same order, 1 three-pass
// order (L1, L2) -> natural, 2 natural -> three-pass order (L1, L2)
template <typename T>
void launch_reorder(const double *in, void *out, int64_t L, int64_t L1, int64_t L2, int mode,
                    hipStream_t s);

// ---- a4 / a6: pack and unpack ----------------------------------------------------
// off / deg (device, per vector, nullable): mixed-degree batches in CSR layout,
// vector b at alpha + off[b] with degree deg[b]; otherwise alpha + b*ld, degree N
// (for mixed batches N is the largest degree).
template <typename T>
void launch_pack(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                 int64_t ld, int64_t N, int64_t batch, void *X /*cpx<T> [batch][nc]*/, int64_t nc,
                 hipStream_t s);
// Wpart2 (may be null with G2 = 0): further partial sums in single precision, from
// the ranks a mixed-precision plan runs in FP32
template <typename T>
void launch_unpack(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                   int64_t ld, double *beta, int64_t N, int64_t batch,
                   const void *Wpart /*cpx<T> [G][batch][nc]*/, int G,
                   const void *Wpart2 /*cpx<float> [G2][batch][nc]*/, int G2, int64_t nc, int64_t L,
                   const double *alias /*launch_alias_sums*/, const double *tsym,
                   const double *row0, hipStream_t s);
// the two plan constants of the circulant alias correction at n - 1 = L/2, from the
// normalised Cholesky columns (zeros when L/2 is not a lane of the plan)
void launch_alias_sums(const double *ell64, int64_t nc_ell, int S, int parts, int64_t L, double *alias,
                       hipStream_t s);
// row 0 by a direct dot product: partial sums over up to ROW0_PMAX workgroups per
// vector into part[batch][ROW0_PMAX], then summed in a fixed order into row0[batch]
constexpr int ROW0_PMAX = 256;
void launch_row0_direct(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                        int64_t ld, int64_t N, int64_t batch, const double *tsym, const double *hk,
                        double *part, double *row0, hipStream_t s);

// variable-length members from device offsets (count + 1 entries): sanitised
// offsets and degrees (-1: skipped; *skipped counts the non-empty ones, may be null)
void launch_varlen(const int64_t *off, int64_t count, int64_t total, int64_t nmax, int64_t *off2, int64_t *deg,
                   int64_t *skipped, hipStream_t s);

// empty kernel k_trace_marker with `id` workgroups of 64 threads (trace regions)
void launch_trace_marker(int id, hipStream_t s);

// ---- static scratch (thx_execute_noalloc) -------------------------------------------
constexpr int64_t SCRATCH_BYTES = (int64_t)512 << 20; // held on every GPU the library runs on
constexpr int SCRATCH_MAX_DEVICES = 64;
// The current device's copy of the scratch (hipGetSymbolAddress once per device,
// with that device current); nullptr and *err set on failure.
void *scratch_device_ptr(hipError_t *err);

// ---- direct O(N^2) ----------------------------------------------------------------
void launch_direct(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                   int64_t ld, double *beta, int64_t N, int64_t batch, const double *tsym,
                   const double *hk, hipStream_t s);
void launch_zero(void *p, int64_t bytes, hipStream_t s);
// I[k][k] = 1 for k < n (row stride ld; the rest must already be zero)
void launch_identity(double *I, int64_t n, int64_t ld, hipStream_t s);

// ---- unit steps: beta = D1 t_0 h_0 (suffix sums of D2 alpha) ----------------------
// tot: suffix_tot_doubles(k, N, batch) doubles of workspace, the totals of the
// SCAN_SPLIT sub-chunks of every chunk (unused for short vectors:
// at most SS_LANES lanes run one wave per vector in one launch, any batch size)
constexpr int SS_LANES = 1024;
constexpr int SCAN_SPLIT = 2;
int suffix_chunks(const KindDesc &k, int64_t N);
inline int64_t suffix_tot_doubles(const KindDesc &k, int64_t N, int64_t batch)
{
    return 2 * SCAN_SPLIT * batch * suffix_chunks(k, N);
}
bool suffix_small(const KindDesc &k, int64_t N);
void launch_suffix(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha, int64_t ld,
                   double *beta, int64_t N, int64_t batch, const double *tsym, const double *hk, double *tot,
                   hipStream_t s);

// ---- dense path: beta_b = A alpha_b with A materialised ----------------------------
// At[k][j] = A[j][k], row-major with stride npad (a multiple of DENSE_PAD), zero
// outside 0..N and for k < j (A upper triangular).  off / deg as for pack.
constexpr int64_t DENSE_PAD = 32;
constexpr int64_t DENSE_MAX = 512;       // largest degree + 1 materialised by default
constexpr int64_t DENSE_TUNE_MAX = 2048; // largest degree + 1 the autotuner tries it for
void launch_dense(const double *At, int64_t npad, const int64_t *off, const int64_t *deg,
                  const double *alpha, int64_t ld, double *beta, int64_t N, int64_t batch,
                  hipStream_t s);
// FP32-bulk plans: the matrix as three bfloat16 parts (dense_bf16_elems(npad)
// 16-bit values, written by launch_split_matrix from At) and the product on the
// bfloat16 matrix cores with FP32 accumulation
int64_t dense_bf16_elems(int64_t npad);
void launch_split_matrix(const double *At, int64_t npad, void *Bp, hipStream_t s);
void launch_dense_bf16(const void *Bp, int64_t npad, const int64_t *off, const int64_t *deg,
                       const double *alpha, int64_t ld, double *beta, int64_t N, int64_t batch,
                       hipStream_t s);

// ---- a5: Toeplitz products ---------------------------------------------------------
// Largest length handled by one workgroup in LDS.  (Twice that, one workgroup
// per CU in 136 KiB, was measured slower than the three passes at every batch
// size.)
template <typename T> constexpr int64_t lds_max_len() { return sizeof(T) == 8 ? 4096 : 8192; }
// Row lengths of the three-pass scheme.  The short row takes half the LDS of
// the long one, so twice as many row workgroups share a CU and the loads,
// transforms and stores of different rows overlap; it is the default while
// the columns stay at most 512 long, where a column tile still spans full
// 128-byte segments.  Longest transform: MP_LMAX.
template <typename T> constexpr int64_t mp_row_short() { return sizeof(T) == 8 ? 2048 : 4096; }
template <typename T> constexpr int64_t mp_row_long() { return sizeof(T) == 8 ? 4096 : 8192; }
// double precision only: rows of 8192 points (one 512-thread workgroup per CU)
// with columns of 256 or 512, so that L = 2^21 and 2^22 keep the 16-column tiles
// of columns of 512 instead of 8-column tiles of columns of 1024
template <typename T> constexpr int64_t mp_row_xl() { return sizeof(T) == 8 ? 8192 : 0; }
constexpr int64_t MP_LMAX = (int64_t)1 << 22;

// single-workgroup path: W[g] = sum_{s in group g} ell_s o IFFT(FFT(ell_s o X) . that),
// largest FFT radix 8 or 16
template <typename T>
bool launch_toep_lds(int64_t L, int radix, const void *X, int64_t nc, int64_t n, const void *ell, int S,
                     int slots_per_group, int G, const void *that, const void *tw, void *Wpart,
                     int64_t batch, hipStream_t s, const AlphaIn *ain = nullptr);
// plain forward FFT of one length-L complex array in LDS (symbol transform), scaled
template <typename T>
bool launch_fft_lds(int64_t L, const void *in, void *out, const void *tw, double scale,
                    hipStream_t s);

struct MultiPassGeom {
    int64_t L, L1, L2, TC;
};
// geometry for length L; `row` selects mp_row_short / mp_row_long, any other
// value (or one that leaves the columns outside 2..1024) the default
template <typename T> MultiPassGeom multipass_geom(int64_t L, int64_t row = 0);
// true when the three-pass kernels are built for rows of L1 points and columns of L / L1
bool multipass_ok(int64_t L, int64_t L1);
// P1: U[s][b] = column FFTs (+ twiddle) of ell_s o X[b] (or of `src` when ell == nullptr),
// `spb` consecutive slots per workgroup; with `ain` the lanes of X are formed from
// the vectors themselves (X unused, no pack step)
template <typename T>
bool launch_mp_p1(const MultiPassGeom &g, const void *X, int64_t nc, int64_t n, const void *ell,
                  int slot0, int nslots, int spb, const void *src, void *U, int64_t batch,
                  const void *twL2, const void *twA, hipStream_t s, const AlphaIn *ain = nullptr);
// P2: row FFT, times permuted symbol, inverse row FFT, conjugate twiddle (full);
// or forward row FFT only, scaled, written to `out` (symbol transform)
template <typename T>
bool launch_mp_p2(const MultiPassGeom &g, void *U, int nslots, int64_t batch, const void *that_perm,
                  const void *twL1, const void *twA, const void *twL2, bool full, void *out,
                  double scale, hipStream_t s);
// P1 and P2 fused for columns of 2 or 4 (false for other geometries): each row
// workgroup forms its row's column DFT directly from ell_s o X, then as P2
template <typename T>
bool launch_mp_p2f(const MultiPassGeom &g, const void *X, int64_t nc, int64_t n, const void *ell, int slot0,
                   int nslots, void *U, int64_t batch, const void *that_perm, const void *twL1, const void *twA,
                   const void *twL2, hipStream_t s);
// P3: inverse column FFTs, scaled by ell_s and summed over the slots of group g
template <typename T>
bool launch_mp_p3(const MultiPassGeom &g, const void *U, int64_t nc, int64_t n, const void *ell,
                  int slot0, int nslots, int slots_per_group, int G, void *Wpart, int gofs,
                  int64_t batch, const void *twL2, hipStream_t s);

} // namespace thx
