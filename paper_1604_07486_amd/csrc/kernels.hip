// kernels.hip -- HIP kernels of libthx for gfx950 (MI355X).
//
// Fig. 1 of the paper, step by step:
//   a1  Lambda / Gamma-ratio tables .................. k_gamma_ratio
//   a2  pivoted Cholesky of the Hankel part(s) ....... k_pchol_init / _select / _column
//   a3  FFT of the embedded Toeplitz symbol .......... k_symbol_embed + FFT kernels
//   a4  v = D2 alpha, packed two real halves per complex lane ... k_pack
//   a5  w = sum_r D_{l_r} T D_{l_r} v via FFTs ....... k_toep_lds / k_mp_p1,p2,p3
//   a6  beta = D1 w (+ circulant alias term, special row) ...... k_unpack, k_row0
// plus the O(N^2) direct evaluation used below the FFT crossover (Sec. 4).
#include "launch.hpp"
#include "fft_reg.hpp"
#include "thx_device.hpp"
#include <math.h>
#include <algorithm>
#include <mutex>

namespace thx {

// ============================================================================
// a1: Gamma-ratio generator
// ============================================================================

__device__ __forceinline__ double gr_series(double w, const GammaRatio &g)
{
    const double u = 1.0 / (w * w);
    double s = g.c[GR_TERMS - 1];
#pragma unroll
    for (int j = GR_TERMS - 2; j >= 0; --j) s = fma(s, u, g.c[j]);
    s *= u;
    double pw;
    if (g.pow_mode == -1) pw = 1.0 / sqrt(w);
    else if (g.pow_mode == 1) pw = sqrt(w);
    else pw = pow(w, g.amb);
    return pw * exp(s);
}

// Gamma(z + a) / Gamma(z + b).  For w = z + (a+b-1)/2 < 12 the argument is
// raised by k steps: R(z) = R(z+k) prod_{i<k} (z+i+b)/(z+i+a).
__device__ double gamma_ratio(double z, const GammaRatio &g)
{
    const double W0 = 12.0;
    const double w = z + 0.5 * (g.a + g.b - 1.0);
    if (w >= W0) return gr_series(w, g);
    const int k = (int)ceil(W0 - w);
    double num = 1.0, den = 1.0;
    for (int i = 0; i < k; ++i) {
        num *= (z + (double)i + g.b);
        den *= (z + (double)i + g.a);
    }
    if (den == 0.0) return HUGE_VAL; // pole of Gamma(z+a)
    if (num == 0.0) return 0.0;      // pole of Gamma(z+b)
    return gr_series(w + (double)k, g) * (num / den);
}

__global__ void k_gamma_ratio(double *out, int64_t count, double z0, GammaRatio g, double scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = scale * gamma_ratio(z0 + (double)i, g);
}

void launch_gamma_ratio(double *out, int64_t count, double z0, const GammaRatio &g, double scale,
                        hipStream_t s)
{
    if (count <= 0) return;
    const int nt = 256;
    k_gamma_ratio<<<(unsigned)((count + nt - 1) / nt), nt, 0, s>>>(out, count, z0, g, scale);
}

// tw[k] = exp(-2 pi i k / M) for k < count, double and (optionally) float
__global__ void k_twiddles(double *tw64, float *tw32, int64_t M, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    double sn, cs;
    sincospi(2.0 * (double)k / (double)M, &sn, &cs);
    tw64[2 * k] = cs;
    tw64[2 * k + 1] = -sn;
    if (tw32) {
        tw32[2 * k] = (float)cs;
        tw32[2 * k + 1] = (float)(-sn);
    }
}

void launch_twiddles(double *tw64, float *tw32, int64_t M, int64_t count, hipStream_t s)
{
    const int nt = 256;
    k_twiddles<<<(unsigned)((count + nt - 1) / nt), nt, 0, s>>>(tw64, tw32, M, count);
}

__global__ void k_cast(const double *in, float *out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (float)in[i];
}

void launch_cast(const double *in, float *out, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    const int nt = 256;
    k_cast<<<(unsigned)((count + nt - 1) / nt), nt, 0, s>>>(in, out, count);
}

// Jacobi diagonal factors (Sec. 5.3, case 2, second parameter b fixed):
//   D1_j = (2j + c) Gamma(j + c) / Gamma(j + b + 1)   (j >= 1),
//   D1_0 = Gamma(c + 1) / Gamma(b + 1)                 (the j = 0 limit, also for c = 0),
//   D2_k = Gamma(k + b + 1) / Gamma(k + e),            c = g + b + 1, e = a + b + 1,
// times (-1)^j when the stage is reflected (P_k^{(a,b)}(-x) = (-1)^k P_k^{(b,a)}(x)),
// and times the Chebyshev normalisation P_j^{(-1/2,-1/2)}(1) = Lambda(j)/sqrt(pi)
// (cheb = 1, applied to D1) or its reciprocal (cheb = 2, applied to D2).
__global__ void k_jacobi_diag(double *out, int64_t count, int which, double c, GammaRatio r1, GammaRatio r0,
                              GammaRatio lam, int reflect, int cheb)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const double z = (double)j;
    double v;
    if (which == 1) v = (j == 0) ? gamma_ratio(0.0, r0) : (2.0 * z + c) * gamma_ratio(z, r1);
    else v = gamma_ratio(z, r1);
    if (reflect && (j & 1)) v = -v;
    const double rsqrtpi = 0.56418958354775628694807945156077259; // 1/sqrt(pi)
    if (cheb == 1) v *= gamma_ratio(z, lam) * rsqrtpi;
    else if (cheb == 2) v /= gamma_ratio(z, lam) * rsqrtpi;
    out[j] = v;
}

void launch_jacobi_diag(double *out, int64_t count, int which, double a, double b, double g, int reflect,
                        int cheb, hipStream_t s)
{
    const double c = g + b + 1.0, e = a + b + 1.0;
    const GammaRatio r1 = which == 1 ? make_gamma_ratio(c, b + 1.0) : make_gamma_ratio(b + 1.0, e);
    const GammaRatio r0 = make_gamma_ratio(c + 1.0, b + 1.0);
    const GammaRatio lam = make_gamma_ratio(0.5, 1.0);
    const int nt = 256;
    k_jacobi_diag<<<(unsigned)((count + nt - 1) / nt), nt, 0, s>>>(out, count, which, c, r1, r0, lam,
                                                                   reflect, cheb);
}

// Jacobi case 3 (a + b <= -1): H_00 and D2_0 hold a 0 * infinity limit; the
// (0, 0) entry of any conversion matrix is 1 (P_0 = 1 in every basis), so set
// h(0) = 1 and D2_0 = 1 / D1_0.
__global__ void k_case3_origin(double *hk, const double *d1, double *d2)
{
    hk[0] = 1.0;
    d2[0] = 1.0 / d1[0];
}
void launch_case3_origin(double *hk, const double *d1, double *d2, hipStream_t s)
{
    k_case3_origin<<<1, 1, 0, s>>>(hk, d1, d2);
}

__global__ void k_set_value(double *p, double v) { *p = v; }
void launch_set_value(double *p, double v, hipStream_t s) { k_set_value<<<1, 1, 0, s>>>(p, v); }

// ============================================================================
// a2: pivoted Cholesky (Sec. 2.1, Fig. 3) of up to two Hankel parts
// ============================================================================
//
// Only the residual diagonal d and the K chosen columns are ever formed.
// Column r of part q (normalised: l~_r = l_r / sqrt(pivot)) is
//   l_r[i] = h(i + p_r) - sum_{m<r} l~_m[i] l~_m[p_r],   l~_r = l_r / sqrt(d[p_r]),
// and d <- d - l~_r^2.  Storage: the normalised columns go to the complex slot
// array `ell`; for two parts, part q is component q of slot r; for one part,
// rank r is component (r & 1) of slot r >> 1.

constexpr int PC_NT = 256;

__device__ __forceinline__ int64_t ell_index(int parts, int q, int r, int64_t i, int64_t nc)
{
    return parts == 2 ? 2 * ((int64_t)r * nc + i) + q : 2 * ((int64_t)(r >> 1) * nc + i) + (r & 1);
}

__device__ __forceinline__ void argmax_merge(double &v, int &i, double v2, int i2)
{
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

// block-wide (max, lowest argmax) of (v, i); result valid in thread 0
__device__ void block_argmax(double &v, int &i, double *sv, int *si)
{
    const int t = threadIdx.x;
    sv[t] = v;
    si[t] = i;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (t < h) {
            double a = sv[t];
            int ai = si[t];
            argmax_merge(a, ai, sv[t + h], si[t + h]);
            sv[t] = a;
            si[t] = ai;
        }
        __syncthreads();
    }
    v = sv[0];
    i = si[0];
}

__device__ __forceinline__ int64_t hk_offset(const PcholArgs &a, int q)
{
    return a.parts == 2 ? q : 0;
}

__global__ __launch_bounds__(PC_NT) void k_pchol_init(PcholArgs a)
{
    __shared__ double sv[PC_NT];
    __shared__ int si[PC_NT];
    const int64_t i = (int64_t)blockIdx.x * PC_NT + threadIdx.x;
    for (int q = 0; q < a.parts; ++q) {
        double v = 0.0;
        if (i < a.nc) {
            double dv = 0.0;
            if (i >= a.a0[q] && i < a.n[q]) dv = a.hk[2 * i + hk_offset(a, q)];
            a.d[q * a.nc + i] = dv;
            v = a.w[q * a.nc + i] * dv;
        }
        int idx = (int)i;
        block_argmax(v, idx, sv, si);
        if (threadIdx.x == 0) {
            a.pv[q * a.nblk + blockIdx.x] = v;
            a.pi[q * a.nblk + blockIdx.x] = idx;
        }
        __syncthreads();
    }
}

// one block: reduce the partial maxima, apply the stopping rule, publish pivot r
__global__ __launch_bounds__(1024) void k_pchol_select(PcholArgs a, int r)
{
    __shared__ double sv[1024];
    __shared__ int si[1024];
    PcholState *st = a.st;
    for (int q = 0; q < a.parts; ++q) {
        if (st->done[q]) {
            if (threadIdx.x == 0) st->active[q] = 0;
            continue;
        }
        double v = -1.0;
        int idx = 0x7fffffff;
        for (int b = threadIdx.x; b < a.nblk; b += blockDim.x)
            argmax_merge(v, idx, a.pv[q * a.nblk + b], a.pi[q * a.nblk + b]);
        block_argmax(v, idx, sv, si);
        __shared__ int go;
        if (threadIdx.x == 0) {
            if (r == 0) st->dmax0[q] = v;
            const double d0 = st->dmax0[q];
            if (r >= a.kcap || !(v > st->eps[q] * d0) || !(v > 0.0)) {
                st->done[q] = 1;
                st->K[q] = r;
                st->dfinal[q] = d0 > 0.0 ? fmax(v, 0.0) / d0 : 0.0;
                st->active[q] = 0;
                go = 0;
            } else {
                st->active[q] = 1;
                st->cur_p[q] = idx;
                st->cur_piv[q] = a.d[q * a.nc + idx]; // unweighted: the Schur step divides by it
                st->piv[q][r] = idx;
                st->pval[q][r] = v;
                go = 1;
            }
        }
        __syncthreads();
        if (go) {
            const int p = st->cur_p[q];
            for (int m = threadIdx.x; m < r; m += blockDim.x)
                st->R[q][r][m] = a.ell[ell_index(a.parts, q, m, p, a.nc)];
        }
        __syncthreads();
    }
}

// Column r of every active part.  The earlier columns are read once per 16-byte
// lane: for two parts, component q of slot m is column m of part q, so one
// pass updates both; for one part, the two components of slot m are its
// columns 2m and 2m + 1.
__global__ __launch_bounds__(PC_NT) void k_pchol_column(PcholArgs a, int r)
{
    __shared__ double sv[PC_NT];
    __shared__ int si[PC_NT];
    const PcholState *st = a.st;
    const int64_t i = (int64_t)blockIdx.x * PC_NT + threadIdx.x;
    const cpx<double> *ec = reinterpret_cast<const cpx<double> *>(a.ell);
    bool act[2], in[2];
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        act[q] = q < a.parts && st->active[q] != 0; // uniform across the grid
        in[q] = act[q] && i < a.nc && i >= a.a0[q] && i < a.n[q];
        if (in[q]) acc[q] = a.hk[i + st->cur_p[q] + hk_offset(a, q)];
    }
    if (a.parts == 2) {
        if (in[0] || in[1]) {
            const double *R0 = st->R[0][r], *R1 = st->R[1][r];
            for (int m = 0; m < r; ++m) {
                const cpx<double> e = ec[(int64_t)m * a.nc + i];
                acc[0] = fma(-e.x, R0[m], acc[0]);
                acc[1] = fma(-e.y, R1[m], acc[1]);
            }
        }
    } else if (in[0]) {
        const double *R0 = st->R[0][r];
        for (int m = 0; 2 * m < r; ++m) {
            const cpx<double> e = ec[(int64_t)m * a.nc + i];
            acc[0] = fma(-e.x, R0[2 * m], acc[0]);
            if (2 * m + 1 < r) acc[0] = fma(-e.y, R0[2 * m + 1], acc[0]);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (!act[q]) continue;
        double dn = 0.0;
        if (i < a.nc) {
            dn = a.d[q * a.nc + i];
            if (in[q]) {
                const double lt = acc[q] / sqrt(st->cur_piv[q]);
                a.ell[ell_index(a.parts, q, r, i, a.nc)] = lt;
                dn = fma(-lt, lt, dn);
                if (!(dn > 0.0) || i == st->cur_p[q]) dn = 0.0;
                a.d[q * a.nc + i] = dn;
            }
            dn *= a.w[q * a.nc + i];
        }
        int idx = (int)i;
        block_argmax(dn, idx, sv, si);
        if (threadIdx.x == 0) {
            a.pv[q * a.nblk + blockIdx.x] = dn;
            a.pi[q * a.nblk + blockIdx.x] = idx;
        }
        __syncthreads();
    }
}

void launch_pchol_init(const PcholArgs &a, hipStream_t s)
{
    k_pchol_init<<<a.nblk, PC_NT, 0, s>>>(a);
}

void launch_pchol_step(const PcholArgs &a, int r, hipStream_t s)
{
    k_pchol_select<<<1, 1024, 0, s>>>(a, r);
    k_pchol_column<<<a.nblk, PC_NT, 0, s>>>(a, r);
}

// ============================================================================
// a3: Toeplitz symbol as the first column of a circulant
// ============================================================================
// y_a = sum_{b >= a} t_{b-a} z_b is the circular correlation with
// e[0] = t_0, e[L-m] = t_m (0 < m < nt), zero elsewhere; then
// y = IFFT(FFT(z) . FFT(e)) restricted to a < n.
__global__ void k_symbol_embed(const double *t, int64_t nt, double *emb, int64_t L)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    double v = 0.0;
    if (i == 0) v = t[0];
    else if (L - i < nt) v = t[L - i];
    emb[2 * i] = v;
    emb[2 * i + 1] = 0.0;
}

void launch_symbol_embed(const double *t, int64_t nt, double *emb, int64_t L, hipStream_t s)
{
    const int nt_ = 256;
    k_symbol_embed<<<(unsigned)((L + nt_ - 1) / nt_), nt_, 0, s>>>(t, nt, emb, L);
}

// Reorder a double-precision spectrum (complex, length L) into the working
// precision.  mode 0: same order; mode 1: from the three-pass order
// in[k2 L1 + k1] to natural order out[k2 + L2 k1]; mode 2: natural order to
// the three-pass order out[k2 L1 + k1] = in[k2 + L2 k1].
template <typename T>
__global__ void k_reorder(const double *in, cpx<T> *out, int64_t L, int64_t L1, int64_t L2, int mode)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    int64_t src = i;
    if (mode == 1) src = (i % L2) * L1 + i / L2;
    else if (mode == 2) src = (i / L1) + L2 * (i % L1);
    out[i] = cpx<T>{(T)in[2 * src], (T)in[2 * src + 1]};
}

template <typename T>
void launch_reorder(const double *in, void *out, int64_t L, int64_t L1, int64_t L2, int mode, hipStream_t s)
{
    const int nt = 256;
    k_reorder<T><<<(unsigned)((L + nt - 1) / nt), nt, 0, s>>>(in, (cpx<T> *)out, L, L1, L2, mode);
}
template void launch_reorder<double>(const double *, void *, int64_t, int64_t, int64_t, int, hipStream_t);
template void launch_reorder<float>(const double *, void *, int64_t, int64_t, int64_t, int, hipStream_t);

// ============================================================================
// Diagonal factors
// ============================================================================

__device__ __forceinline__ double d1_of(const KindDesc &k, int64_t j)
{
    if (k.d1tab) return k.d1tab[j];
    switch (k.kind) {
    case 0: return j == 0 ? M_1_PI : M_2_PI;           // leg2cheb: (2/pi) diag(1/2, 1, ...)
    case 1: return (double)j + 0.5;                    // cheb2leg: diag(j + 1/2)
    case 2: return (double)j + k.p[1];                 // ultra: diag(j + lambda2)
    default: return 1.0;
    }
}

__device__ __forceinline__ double d2_of(const KindDesc &k, int64_t j)
{
    if (k.d2tab) return k.d2tab[j];
    if (k.kind == 1) return j == 0 ? -0.5641895835477562869480795 /* -1/sqrt(pi) */ : -0.25 * (double)j;
    return 1.0;
}

// ============================================================================
// a4: pack v = D2 alpha into complex lanes
// ============================================================================
// parity-split kinds: lane a holds (v_{2a}, v_{2a+1}); otherwise (v_a, v_a).
// Per-vector addressing: fixed-degree batches use alpha + b*ld with degree N;
// mixed-degree batches pass member offsets / degrees (CSR layout).
struct VecRef {
    const int64_t *off; // nullable
    const int64_t *deg; // nullable
};
__device__ __forceinline__ void vec_of(const VecRef &v, int64_t b, int64_t ld, int64_t N, int64_t &base,
                                       int64_t &n)
{
    if (v.off) {
        base = v.off[b];
        n = v.deg[b];
    } else {
        base = b * ld;
        n = N;
    }
}

template <typename T>
__global__ void k_pack(KindDesc k, VecRef vr, const double *alpha, int64_t ld, int64_t N0, cpx<T> *X,
                       int64_t nc)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (a >= nc) return;
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    const double *al = alpha + base;
    double x = 0.0, y = 0.0;
    if (k.parity) {
        const int64_t j0 = 2 * a, j1 = 2 * a + 1;
        if (j0 <= N) x = d2_of(k, j0) * al[j0];
        if (j1 <= N) y = d2_of(k, j1) * al[j1];
    } else if (a <= N) {
        x = y = d2_of(k, a) * al[a];
    }
    X[b * nc + a] = cpx<T>{(T)x, (T)y};
}

// lane a of a vector (base pointer al, degree N) as k_pack forms it, in precision T
template <typename T>
__device__ __forceinline__ cpx<T> x_lane(const KindDesc &k, const double *al, int64_t N, int64_t a)
{
    double x = 0.0, y = 0.0;
    if (k.parity && 2 * a + 1 <= N && ((uintptr_t)(al + 2 * a) & 15) == 0) {
        const double2 v = *(const double2 *)(al + 2 * a); // both inside the vector: one 16-byte load
        x = d2_of(k, 2 * a) * v.x;
        y = d2_of(k, 2 * a + 1) * v.y;
    } else if (k.parity) {
        const int64_t j0 = 2 * a, j1 = 2 * a + 1;
        if (j0 <= N) x = d2_of(k, j0) * al[j0];
        if (j1 <= N) y = d2_of(k, j1) * al[j1];
    } else if (a <= N) {
        x = y = d2_of(k, a) * al[a];
    }
    return cpx<T>{(T)x, (T)y};
}

template <typename T>
void launch_pack(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                 int64_t ld, int64_t N, int64_t batch, void *X, int64_t nc, hipStream_t s)
{
    const int nt = 256;
    dim3 grid((unsigned)((nc + nt - 1) / nt), (unsigned)batch);
    k_pack<T><<<grid, nt, 0, s>>>(k, VecRef{off, deg}, alpha, ld, N, (cpx<T> *)X, nc);
}
template void launch_pack<double>(const KindDesc &, const int64_t *, const int64_t *, const double *, int64_t, int64_t, int64_t, void *, int64_t, hipStream_t);
template void launch_pack<float>(const KindDesc &, const int64_t *, const int64_t *, const double *, int64_t, int64_t, int64_t, void *, int64_t, hipStream_t);

// ============================================================================
// a2 (continued): pivot weights and stopping threshold of the pivoted Cholesky
// ============================================================================
// The truncation error of A = D1 (T o H) D2 is D1 (T o E) D2 alpha with E the
// PSD residual of H, |E_jk| <= sqrt(E_jj E_kk).  Writing w_j = |D1_j D2_j| and
// r_j = sqrt|D1_j / D2_j|, |D1_j| sqrt(E_jj) = r_j sqrt(w_j E_jj) and
// |D2_k| sqrt(E_kk) = sqrt(w_k E_kk) / r_k, so
//   |beta error_j| <= Tmax amp max_i(w_i E_ii) ||alpha||_1,  amp = max_{j<=k} r_j / r_k.
// Pivoting on w_i d_i is the diagonal pivoting of S H S, S = diag(sqrt w): it
// removes first the residual that D1 and D2 amplify most.  Stopping once
// max w_i d_i <= eps max w_i H_ii with eps = 2 tol |t_0| / (amp Tmax) bounds the
// error by 2 tol max_j |A_jj| ||alpha||_1 (max w_i H_ii |t_0| = max |A_jj|).

// lane i of part q holds coefficient j = 2i + q (parity-split kinds) or j = i
__device__ __forceinline__ int64_t part_index(const KindDesc &k, int q, int64_t i)
{
    return k.parity ? 2 * i + q : i;
}

__global__ void k_pchol_w(KindDesc k, PcholArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nc) return;
    for (int q = 0; q < a.parts; ++q) {
        double w = 0.0;
        if (i >= a.a0[q] && i < a.n[q]) {
            const int64_t j = part_index(k, q, i);
            w = fabs(d1_of(k, j) * d2_of(k, j));
            if (!(w < INFINITY)) w = 0.0; // also NaN
        }
        a.w[q * a.nc + i] = w;
    }
}

constexpr int AMP_NT = 1024;

__device__ __forceinline__ double amp_r(const KindDesc &k, const PcholArgs &a, int q, int64_t i)
{
    if (!(a.w[q * a.nc + i] > 0.0)) return 0.0; // outside the part, or a zero factor
    const int64_t j = part_index(k, q, i);
    return sqrt(fabs(d1_of(k, j) / d2_of(k, j)));
}

__device__ double block_max(double v, double *sv)
{
    const int t = threadIdx.x;
    sv[t] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (t < h) sv[t] = fmax(sv[t], sv[t + h]);
        __syncthreads();
    }
    const double m = sv[0];
    __syncthreads();
    return m;
}

__global__ __launch_bounds__(AMP_NT) void k_pchol_amp(KindDesc k, PcholArgs a, const double *tsym, int64_t nt,
                                                      double tol, double floor_rel)
{
    __shared__ double sv[AMP_NT];
    __shared__ double pre[AMP_NT];
    const int t = threadIdx.x;
    // Tmax and |t_0| of the Toeplitz symbol
    double tm = 0.0;
    for (int64_t m = t; m < nt; m += AMP_NT) tm = fmax(tm, fabs(tsym[m]));
    const double Tmax = block_max(tm, sv);
    const double t0 = fabs(tsym[0]) > 0.0 ? fabs(tsym[0]) : Tmax;
    for (int q = 0; q < a.parts; ++q) {
        // amp = max over i <= i' of r_i / r_i' (indices with w > 0): chunked, with an
        // exclusive prefix maximum of the chunk maxima
        const int64_t lo = a.a0[q], hi = a.n[q];
        const int64_t len = hi > lo ? hi - lo : 0;
        const int64_t C = (len + AMP_NT - 1) / AMP_NT;
        const int64_t c0 = lo + (int64_t)t * C, c1 = c0 + C < hi ? c0 + C : hi;
        double cm = 0.0;
        for (int64_t i = c0; i < c1; ++i) cm = fmax(cm, amp_r(k, a, q, i));
        pre[t] = cm;
        __syncthreads();
        if (t == 0) {
            double run = 0.0;
            for (int u = 0; u < AMP_NT; ++u) {
                const double x = pre[u];
                pre[u] = run;
                run = fmax(run, x);
            }
        }
        __syncthreads();
        double run = pre[t], best = 0.0;
        for (int64_t i = c0; i < c1; ++i) {
            const double r = amp_r(k, a, q, i);
            if (!(r > 0.0)) continue;
            run = fmax(run, r);
            best = fmax(best, run / r);
        }
        const double amp = fmax(block_max(best, sv), 1e-300);
        if (t == 0) {
            const double e = Tmax > 0.0 ? 2.0 * tol * t0 / (amp * Tmax) : tol;
            a.st->eps[q] = fmax(e, floor_rel);
            a.st->escale[q] = Tmax > 0.0 ? amp * Tmax / (2.0 * t0) : 1.0;
        }
        __syncthreads();
    }
}

void launch_pchol_weights(const KindDesc &k, const PcholArgs &a, const double *tsym, int64_t nt, double tol,
                          double floor_rel, hipStream_t s)
{
    k_pchol_w<<<(unsigned)((a.nc + 255) / 256), 256, 0, s>>>(k, a);
    k_pchol_amp<<<1, AMP_NT, 0, s>>>(k, a, tsym, nt, tol, floor_rel);
}

// ============================================================================
// a6: sum the partial results, remove the circulant alias, beta = D1 w
// ============================================================================
// When L = 2n - 2 for a half of size n, the correlation picks up exactly one
// extra term t_{n-1} z_0 at output n-1; it is removed here in double precision:
//   w_{n-1} -= t_{n-1} v_0 sum_s l~_s[n-1] l~_s[0].
// One thread per complex lane: parity kinds write both halves' outputs
// (2a, 2a + 1) of lane a, the others output a (the sum of its two packed
// ranks).  The G partial results are loaded four at a time and added in
// group order.
// The alias term only arises for n - 1 = L/2, so its factor is a plan constant:
// alias[q] = sum_s l~_s[L/2].q l~_s[0].q for the two parts of the parity kinds,
// alias[0] = sum_s (both packed ranks of slot s) otherwise, summed in slot order.
__global__ __launch_bounds__(KMAX) void k_alias_sums(const double *ell64, int64_t nc_ell, int S, int parts,
                                                     int64_t idx, double *alias)
{
    __shared__ double pr[2][KMAX];
    const int s = threadIdx.x;
    if (s < S) {
        const double *e = ell64 + 2 * ((int64_t)s * nc_ell + idx), *o = ell64 + 2 * ((int64_t)s * nc_ell);
        pr[0][s] = e[0] * o[0];
        pr[1][s] = e[1] * o[1];
    }
    __syncthreads();
    if (s == 0) {
        double g0 = 0.0, g1 = 0.0;
        for (int t = 0; t < S; ++t) {
            if (parts == 2) {
                g0 += pr[0][t];
                g1 += pr[1][t];
            } else {
                g0 += pr[0][t];
                g0 += pr[1][t];
            }
        }
        alias[0] = g0;
        alias[1] = g1;
    }
}

void launch_alias_sums(const double *ell64, int64_t nc_ell, int S, int parts, int64_t L, double *alias,
                       hipStream_t s)
{
    if (S < 1 || S > KMAX || L / 2 >= nc_ell) {
        launch_zero(alias, 2 * (int64_t)sizeof(double), s); // the alias position is never an output
        return;
    }
    k_alias_sums<<<1, KMAX, 0, s>>>(ell64, nc_ell, S, parts, L / 2, alias);
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(KindDesc k, VecRef vr, const double *alpha, int64_t ld,
                                                double *beta, int64_t N0, const cpx<T> *W, int G,
                                                const cpx<float> *W2, int G2, int64_t nc,
                                                int64_t batch, int64_t L, const double *alias,
                                                const double *tsym, const double *row0)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    if (a > (k.parity ? N / 2 : N)) return;
    const double *al = alpha + base;
    const cpx<T> *Wa = W + b * nc + a;
    const int64_t gstride = batch * nc;
    double wx = 0.0, wy = 0.0, wsum = 0.0;
    int g = 0;
    // eight partial groups in flight per round (the sum keeps the group order)
    for (; g + 8 <= G; g += 8) {
        cpx<T> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = Wa[(int64_t)(g + u) * gstride];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            wx += (double)v[u].x;
            wy += (double)v[u].y;
            wsum += (double)v[u].x + (double)v[u].y;
        }
    }
    for (; g + 4 <= G; g += 4) {
        cpx<T> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = Wa[(int64_t)(g + u) * gstride];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            wx += (double)v[u].x;
            wy += (double)v[u].y;
            wsum += (double)v[u].x + (double)v[u].y;
        }
    }
    for (; g < G; ++g) {
        const cpx<T> v = Wa[(int64_t)g * gstride];
        wx += (double)v.x;
        wy += (double)v.y;
        wsum += (double)v.x + (double)v.y;
    }
    if (G2 > 0) {
        const cpx<float> *W2a = W2 + b * nc + a;
        for (g = 0; g < G2; ++g) {
            const cpx<float> v = W2a[(int64_t)g * gstride];
            wx += (double)v.x;
            wy += (double)v.y;
            wsum += (double)v.x + (double)v.y;
        }
    }
    if (k.parity) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t j = 2 * a + q;
            if (j > N) break;
            double w = q ? wy : wx;
            const int64_t nq = q ? (N + 1) / 2 : N / 2 + 1;
            if (2 * nq - 2 == L && a == nq - 1) w -= tsym[nq - 1] * alias[q] * (d2_of(k, q) * al[q]);
            double out = d1_of(k, j) * w;
            if (row0 && j == 0) out = row0[b];
            beta[base + j] = out;
        }
    } else {
        const int64_t j = a, n = N + 1;
        double w = wsum;
        if (2 * n - 2 == L && j == n - 1) w -= tsym[n - 1] * alias[0] * (d2_of(k, 0) * al[0]);
        double out = d1_of(k, j) * w;
        if (row0 && j == 0) out = row0[b];
        beta[base + j] = out;
    }
}

template <typename T>
void launch_unpack(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                   int64_t ld, double *beta, int64_t N, int64_t batch, const void *Wpart, int G,
                   const void *Wpart2, int G2, int64_t nc, int64_t L, const double *alias,
                   const double *tsym, const double *row0, hipStream_t s)
{
    const int nt = 256;
    const int64_t lanes = k.parity ? N / 2 + 1 : N + 1;
    dim3 grid((unsigned)((lanes + nt - 1) / nt), (unsigned)batch);
    k_unpack<T><<<grid, nt, 0, s>>>(k, VecRef{off, deg}, alpha, ld, beta, N, (const cpx<T> *)Wpart, G,
                                    (const cpx<float> *)Wpart2, Wpart2 ? G2 : 0, nc, batch, L, alias, tsym,
                                    row0);
}
template void launch_unpack<double>(const KindDesc &, const int64_t *, const int64_t *, const double *, int64_t, double *, int64_t, int64_t, const void *, int, const void *, int, int64_t, int64_t, const double *, const double *, const double *, hipStream_t);
template void launch_unpack<float>(const KindDesc &, const int64_t *, const int64_t *, const double *, int64_t, double *, int64_t, int64_t, const void *, int, const void *, int, int64_t, int64_t, const double *, const double *, const double *, hipStream_t);

// Row 0 computed directly when the Hankel part is PSD only on indices >= 1
// (cheb2leg, Sec. 5.1; Jacobi case 3, Sec. 5.3): rows/columns >= 1 go through
// the low-rank path and
//   beta_0 = D1_0 sum_k t_k h(k) D2_k alpha_k   (k even only for parity kinds),
// with the (0, 0) entry set through h(0), D2_0 by the plan.
// Row 0 is a dot product of length N/2+1 (parity kinds) or N+1; it is split
// over P workgroups per vector whose partial sums are then added in a fixed
// order (deterministic, and fast at large N where one workgroup would stream
// the tables alone).
__global__ __launch_bounds__(256) void k_row0_part(KindDesc k, VecRef vr, const double *alpha, int64_t ld,
                                                   int64_t N0, const double *tsym, const double *hk,
                                                   int64_t chunk, double *part)
{
    __shared__ double sm[256];
    const int64_t b = blockIdx.y;
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    const double *al = alpha + base;
    const int64_t cmax = N < 0 ? -1 : (k.parity ? N / 2 : N); // last term index (none: empty vector)
    const int64_t c0 = (int64_t)blockIdx.x * chunk, c1 = min(cmax + 1, c0 + chunk);
    double acc = 0.0;
    if (k.parity) {
        for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x)
            acc = fma(tsym[c] * hk[c], d2_of(k, 2 * c) * al[2 * c], acc);
    } else {
        for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x)
            acc = fma(tsym[c] * hk[c], d2_of(k, c) * al[c], acc);
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * ROW0_PMAX + blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(ROW0_PMAX) void k_row0_sum(KindDesc k, const double *part, int P, double *row0)
{
    __shared__ double sm[ROW0_PMAX];
    const int64_t b = blockIdx.x;
    sm[threadIdx.x] = (int)threadIdx.x < P ? part[b * ROW0_PMAX + threadIdx.x] : 0.0;
    __syncthreads();
    for (int h = ROW0_PMAX / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) row0[b] = d1_of(k, 0) * sm[0];
}

void launch_row0_direct(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                        int64_t ld, int64_t N, int64_t batch, const double *tsym, const double *hk,
                        double *part, double *row0, hipStream_t s)
{
    const int64_t terms = (k.parity ? N / 2 : N) + 1;
    const int64_t P = std::min<int64_t>(ROW0_PMAX, std::max<int64_t>(1, (terms + 2047) / 2048));
    const int64_t chunk = (terms + P - 1) / P;
    k_row0_part<<<dim3((unsigned)P, (unsigned)batch), 256, 0, s>>>(k, VecRef{off, deg}, alpha, ld, N, tsym, hk,
                                                                  chunk, part);
    k_row0_sum<<<(unsigned)batch, ROW0_PMAX, 0, s>>>(k, part, (int)P, row0);
}

// An empty kernel that marks a point in a kernel trace (its grid has `id`
// workgroups of 64 threads, so the trace shows id * 64 as the grid size).
__global__ void k_trace_marker() {}
void launch_trace_marker(int id, hipStream_t s) { k_trace_marker<<<(unsigned)id, 64, 0, s>>>(); }

// Per-member degrees of a variable-length execution from device offsets:
// member i is alpha[off[i] .. off[i+1]-1].  Members that are malformed, reach
// beyond `total` or exceed the plan's degree are skipped (degree -1, nothing
// read or written) and counted in *skipped when it is given; empty members are
// skipped silently.
__global__ void k_varlen(const int64_t *off, int64_t count, int64_t total, int64_t nmax, int64_t *off2,
                         int64_t *deg, unsigned long long *skipped)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t o0 = off[i], o1 = off[i + 1], n = o1 - o0 - 1;
    const bool ok = o0 >= 0 && o1 <= total && n >= 0 && n <= nmax;
    off2[i] = ok ? o0 : 0;
    deg[i] = ok ? n : -1;
    if (!ok && n != -1 && skipped) atomicAdd(skipped, 1ull);
}

void launch_varlen(const int64_t *off, int64_t count, int64_t total, int64_t nmax, int64_t *off2, int64_t *deg,
                   int64_t *skipped, hipStream_t s)
{
    const int nt = 256;
    k_varlen<<<(unsigned)((count + nt - 1) / nt), nt, 0, s>>>(off, count, total, nmax, off2, deg,
                                                               (unsigned long long *)skipped);
}

// ============================================================================
// Static scratch of thx_execute_noalloc: every workspace buffer of such an
// execution is carved from this array, so the call allocates nothing.  Each GPU
// holds its own copy at its own address; host code must use the address from
// hipGetSymbolAddress (the array's name is a host-side stand-in).
// ============================================================================
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

void *scratch_device_ptr(hipError_t *err)
{
    static std::mutex mu;
    static void *ptrs[SCRATCH_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= SCRATCH_MAX_DEVICES)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)); // with `dev` current: that GPU's copy
        if (e != hipSuccess || !q) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        ptrs[dev] = q;
    }
    *err = hipSuccess;
    return ptrs[dev];
}

// ============================================================================
// Direct O(N^2) evaluation (Sec. 4 "Direct"): entries generated on the fly
// ============================================================================
__global__ void k_direct(KindDesc k, VecRef vr, const double *alpha, int64_t ld, double *beta,
                         int64_t N0, const double *tsym, const double *hk)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    if (j > N) return;
    const double *al = alpha + base;
    double acc = 0.0;
    const int64_t cend = k.band >= 0 ? min(N, j + k.band) : N;
    if (k.parity) {
        for (int64_t c = j; c <= cend; c += 2)
            acc = fma(tsym[(c - j) >> 1] * hk[(j + c) >> 1], d2_of(k, c) * al[c], acc);
    } else {
        for (int64_t c = j; c <= cend; ++c) acc = fma(tsym[c - j] * hk[j + c], d2_of(k, c) * al[c], acc);
    }
    beta[base + j] = d1_of(k, j) * acc;
}

void launch_direct(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha,
                   int64_t ld, double *beta, int64_t N, int64_t batch, const double *tsym,
                   const double *hk, hipStream_t s)
{
    const int nt = 128;
    dim3 grid((unsigned)((N + 1 + nt - 1) / nt), (unsigned)batch);
    k_direct<<<grid, nt, 0, s>>>(k, VecRef{off, deg}, alpha, ld, beta, N, tsym, hk);
}

// zero fill (used instead of a memset node so that launch sequences can be graph-captured)
__global__ void k_zero(double *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}
void launch_zero(void *p, int64_t bytes, hipStream_t s)
{
    const int64_t count = bytes / 8;
    if (count <= 0) return;
    k_zero<<<(unsigned)((count + 255) / 256), 256, 0, s>>>((double *)p, count);
}

__global__ void k_identity(double *I, int64_t n, int64_t ld)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) I[k * ld + k] = 1.0;
}
void launch_identity(double *I, int64_t n, int64_t ld, hipStream_t s)
{
    if (n <= 0) return;
    k_identity<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(I, n, ld);
}

// ============================================================================
// Unit steps (case 1): a parameter lowered by exactly 1 makes T and H constant,
// so beta_j = D1_j t_0 h_0 sum_{k >= j, k - j in the kind's stride} D2_k alpha_k:
// a suffix sum, computed as a reverse scan in FP64.  Each partial sum then
// carries rounding relative to its own terms (an FFT's error is relative to
// the largest term of the whole vector, which D1_j ~ j^(first+1) amplifies).
// Parity kinds scan the even and odd indices together as the two components
// of a lane (lane q = indices 2q, 2q+1); other kinds scan every index.
// Pass 1: totals of sub-chunks; pass 2: reverse scan of each chunk of SC_CH
// lanes plus the sum of all later sub-chunks (fixed order: deterministic).
// ============================================================================
constexpr int SC_NT = 256, SC_PER = 4, SC_CH = SC_NT * SC_PER;

// (D2 alpha) at the two components of lane q (returned by value: conditional
// writes through references made the compiler keep the pair in scratch memory)
struct Pair {
    double x, y;
};
__device__ __forceinline__ Pair sc_lane(const KindDesc &k, const double *al, int64_t N, int64_t q)
{
    if (k.parity) {
        const int64_t j0 = 2 * q, j1 = 2 * q + 1;
        const double x = j0 <= N ? d2_of(k, j0) * al[j0] : 0.0;
        const double y = j1 <= N ? d2_of(k, j1) * al[j1] : 0.0;
        return Pair{x, y};
    }
    return Pair{q <= N ? d2_of(k, q) * al[q] : 0.0, 0.0};
}

// The same values with one 16-byte load per lane when the vector's first
// coefficient is 16-byte aligned (a16, uniform per vector) and the lane lies
// inside the vector (the two 8-byte loads of sc_lane touch every cache line
// twice).
__device__ __forceinline__ Pair sc_lane_v(const KindDesc &k, const double *al, int64_t N, int64_t q, bool a16)
{
    if (k.parity && a16 && 2 * q + 1 <= N) {
        const double2 v = *(const double2 *)(al + 2 * q);
        return Pair{d2_of(k, 2 * q) * v.x, d2_of(k, 2 * q + 1) * v.y};
    }
    return sc_lane(k, al, N, q);
}

// beta at the components of lane q: D1 g times the scanned values, one 16-byte
// store per lane under the same conditions as sc_lane_v
__device__ __forceinline__ void sc_store(const KindDesc &k, double *be, int64_t N, int64_t q, double g, double vx,
                                         double vy, bool a16)
{
    if (k.parity) {
        const int64_t j0 = 2 * q, j1 = 2 * q + 1;
        if (a16 && j1 <= N) {
            *(double2 *)(be + j0) = double2{d1_of(k, j0) * g * vx, d1_of(k, j1) * g * vy};
        } else {
            if (j0 <= N) be[j0] = d1_of(k, j0) * g * vx;
            if (j1 <= N) be[j1] = d1_of(k, j1) * g * vy;
        }
    } else if (q <= N) {
        be[q] = d1_of(k, q) * g * vx;
    }
}

// Sums in a fixed order (deterministic): within a wave by butterfly shuffles,
// across the SC_NT / 64 waves through LDS.
constexpr int SC_NW = SC_NT / 64;
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// sum of v over the lanes >= this lane of the wave
__device__ __forceinline__ double wave_suffix(double v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_down(v, o, 64);
        if (lane + o < 64) v += u;
    }
    return v;
}
__device__ __forceinline__ void block_sum2(double &x, double &y, double *sx, double *sy)
{
    x = wave_sum(x);
    y = wave_sum(y);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sx[w] = x;
        sy[w] = y;
    }
    __syncthreads();
    x = 0.0;
    y = 0.0;
#pragma unroll
    for (int i = 0; i < SC_NW; ++i) {
        x += sx[i];
        y += sy[i];
    }
    __syncthreads();
}

// Global memory is read and written with consecutive lanes on consecutive
// threads; the chunk goes through LDS so that each thread can scan a run of
// SC_PER consecutive lanes.
// Pass 1 sums sub-chunks of SC_CH / SC_SPLIT lanes, pass 2 adds the totals of the
// sub-chunks after its chunk.  Short workgroups measured faster in both passes
// (64 vectors of 2^18 + 1 coefficients, parity kind: pass 1 over 2048 / 1024 /
// 512 lanes 43 / 37 / 35 us, pass 2 over 2048 / 1024 / 512 lanes 59 / 50 / 61 us).
constexpr int SC_SPLIT = SCAN_SPLIT, SC_SUBPER = SC_PER / SC_SPLIT;
static_assert(SC_SUBPER * SC_SPLIT == SC_PER, "sub-chunks");
__global__ __launch_bounds__(SC_NT) void k_suffix_tot(KindDesc k, VecRef vr, const double *alpha, int64_t ld,
                                                      int64_t N0, double *tot, int nsub)
{
    __shared__ double sx[SC_NW], sy[SC_NW];
    const int c = blockIdx.x;
    const int64_t b = blockIdx.y;
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    const double *al = alpha + base;
    const bool a16 = ((uintptr_t)al & 15) == 0;
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int i = 0; i < SC_SUBPER; ++i) {
        const Pair u = sc_lane_v(k, al, N, (int64_t)c * (SC_CH / SC_SPLIT) + threadIdx.x + SC_NT * i, a16);
        x += u.x;
        y += u.y;
    }
    block_sum2(x, y, sx, sy);
    if (threadIdx.x == 0) {
        tot[2 * (b * nsub + c)] = x;
        tot[2 * (b * nsub + c) + 1] = y;
    }
}

// LDS index of chunk lane i, padded one slot per 32 against bank conflicts of
// the per-thread runs
__device__ __forceinline__ int sc_pad(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(SC_NT) void k_suffix_apply(KindDesc k, VecRef vr, const double *alpha, int64_t ld,
                                                        double *beta, int64_t N0, const double *tot, int nchunk,
                                                        const double *tsym, const double *hk)
{
    constexpr int LP = SC_CH + SC_CH / 32;
    __shared__ double lx[LP], ly[LP];
    __shared__ double sx[SC_NW], sy[SC_NW];
    const int c = blockIdx.x;
    const int64_t b = blockIdx.y;
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    const int64_t nl = k.parity ? N / 2 + 1 : N + 1; // lanes of this vector
    if ((int64_t)c * SC_CH >= nl) return;            // uniform over the block
    const double *al = alpha + base;
    double *be = beta + base;
    const bool a16 = (((uintptr_t)al | (uintptr_t)be) & 15) == 0;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t q0 = (int64_t)c * SC_CH;
#pragma unroll
    for (int i = 0; i < SC_PER; ++i) {
        const Pair u = sc_lane_v(k, al, N, q0 + t + SC_NT * i, a16);
        lx[sc_pad(t + SC_NT * i)] = u.x;
        ly[sc_pad(t + SC_NT * i)] = u.y;
    }
    // carry: everything after this chunk
    double cx = 0.0, cy = 0.0;
    const int nsub = SC_SPLIT * nchunk;
    for (int cc = SC_SPLIT * (c + 1) + t; cc < nsub; cc += SC_NT) {
        cx += tot[2 * (b * nsub + cc)];
        cy += tot[2 * (b * nsub + cc) + 1];
    }
    block_sum2(cx, cy, sx, sy); // also orders the LDS stores above before the reads below
    // reverse inclusive scan of this thread's run of SC_PER lanes
    double vx[SC_PER], vy[SC_PER];
    double rx = 0.0, ry = 0.0;
#pragma unroll
    for (int i = SC_PER - 1; i >= 0; --i) {
        rx += lx[sc_pad(t * SC_PER + i)];
        ry += ly[sc_pad(t * SC_PER + i)];
        vx[i] = rx;
        vy[i] = ry;
    }
    // exclusive reverse scan of the run totals: within the wave by shuffles,
    // then the totals of the later waves
    const double ix = wave_suffix(rx), iy = wave_suffix(ry);
    double ex = __shfl_down(ix, 1, 64), ey = __shfl_down(iy, 1, 64);
    if (lane == 63) ex = ey = 0.0;
    if (lane == 0) {
        sx[w] = ix;
        sy[w] = iy;
    }
    __syncthreads();
    for (int w2 = w + 1; w2 < SC_NW; ++w2) {
        ex += sx[w2];
        ey += sy[w2];
    }
    ex += cx;
    ey += cy;
#pragma unroll
    for (int i = 0; i < SC_PER; ++i) {
        lx[sc_pad(t * SC_PER + i)] = vx[i] + ex;
        ly[sc_pad(t * SC_PER + i)] = vy[i] + ey;
    }
    __syncthreads();
    const double g = tsym[0] * hk[0];
#pragma unroll
    for (int i = 0; i < SC_PER; ++i) {
        const int li = t + SC_NT * i;
        sc_store(k, be, N, q0 + li, g, lx[sc_pad(li)], ly[sc_pad(li)], a16);
    }
}

int suffix_chunks(const KindDesc &k, int64_t N)
{
    const int64_t nl = k.parity ? N / 2 + 1 : N + 1;
    return (int)((nl + SC_CH - 1) / SC_CH);
}

// Short vectors (at most SS_LANES lanes): one wave per vector, one launch.  Lane
// q of the vector goes to thread q % 64 in run q / 64 (coalesced loads and
// stores).  The runs are taken from the last down: each is reverse-scanned by
// wave shuffles and gets the total of the later runs as a carry (fixed order:
// deterministic); the next run's values are loaded while the current one is
// scanned.
constexpr int SS_NT = 256;

__global__ __launch_bounds__(SS_NT) void k_suffix_small(KindDesc k, VecRef vr, const double *alpha, int64_t ld,
                                                       double *beta, int64_t N0, int64_t batch,
                                                       const double *tsym, const double *hk)
{
    const int t = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (SS_NT / 64) + (threadIdx.x >> 6);
    if (b >= batch) return; // uniform over the wave
    int64_t base, N;
    vec_of(vr, b, ld, N0, base, N);
    if (N < 0) return;
    const int64_t nl = k.parity ? N / 2 + 1 : N + 1;
    const int R = (int)((nl + 63) / 64);
    const double *al = alpha + base;
    double *be = beta + base;
    const bool a16 = (((uintptr_t)al | (uintptr_t)be) & 15) == 0;
    const double g = tsym[0] * hk[0];
    double cx = 0.0, cy = 0.0;
    Pair u = sc_lane_v(k, al, N, (int64_t)(R - 1) * 64 + t, a16);
    for (int i = R - 1; i >= 0; --i) {
        const Pair nxt = i > 0 ? sc_lane_v(k, al, N, (int64_t)(i - 1) * 64 + t, a16) : Pair{0.0, 0.0};
        const double sx = wave_suffix(u.x), sy = wave_suffix(u.y);
        sc_store(k, be, N, (int64_t)i * 64 + t, g, sx + cx, sy + cy, a16);
        cx += __shfl(sx, 0, 64);
        cy += __shfl(sy, 0, 64);
        u = nxt;
    }
}

bool suffix_small(const KindDesc &k, int64_t N) { return (k.parity ? N / 2 + 1 : N + 1) <= SS_LANES; }

void launch_suffix(const KindDesc &k, const int64_t *off, const int64_t *deg, const double *alpha, int64_t ld,
                   double *beta, int64_t N, int64_t batch, const double *tsym, const double *hk, double *tot,
                   hipStream_t s)
{
    if (suffix_small(k, N)) {
        const int64_t blocks = (batch + SS_NT / 64 - 1) / (SS_NT / 64);
        k_suffix_small<<<(unsigned)blocks, SS_NT, 0, s>>>(k, VecRef{off, deg}, alpha, ld, beta, N, batch, tsym, hk);
        return;
    }
    const int nchunk = suffix_chunks(k, N);
    dim3 grid((unsigned)nchunk, (unsigned)batch);
    k_suffix_tot<<<dim3((unsigned)(SC_SPLIT * nchunk), (unsigned)batch), SC_NT, 0, s>>>(
        k, VecRef{off, deg}, alpha, ld, N, tot, SC_SPLIT * nchunk);
    k_suffix_apply<<<grid, SC_NT, 0, s>>>(k, VecRef{off, deg}, alpha, ld, beta, N, tot, nchunk, tsym, hk);
}

// ============================================================================
// Dense path (short vectors): beta_b = A alpha_b as one batched product
// ============================================================================
// The matrix is an O(N^2) object anyway below the FFT crossover; materialised
// once per plan, every execution is a contraction over k on the matrix cores:
//   C[b][j] = sum_k alpha[b][k] At[k][j],   At[k][j] = A[j][k] = 0 for k < j.
// Workgroup: 64 vectors x one chunk of up to 256 (or 64) outputs; wave w owns
// vectors 16w..16w+15 and all 16-column output tiles of the chunk, so every
// wave has the same (triangular) work between two barriers.  Chunks of 16 k of
// both operands go through LDS; the next chunk is read into registers while
// the matrix cores work on the current one.
// v_mfma_f64_16x16x4f64 lane layout: operand a = X[m = lane&15][k = lane>>4],
// operand b = Y[k = lane>>4][n = lane&15], result element i of a lane is
// D[(lane>>4) + 4i][lane&15].
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int DN_BK = 16, DN_NT = 256;
constexpr int DN_XW = DN_BK + 1;                // alpha tile row stride (doubles)
static_assert(DENSE_PAD % DN_BK == 0, "dense tiling");

// BN outputs per workgroup: 256, or 64 when there are too few vectors to give
// every CU a workgroup of 256 outputs.  BM vectors per workgroup: 64 (wave w
// owns vectors 16w..16w+15 and every output tile), or 32 (two waves per group of
// 16 vectors, each taking every other output tile, so both keep the same
// triangular share).  Compiled for three waves per SIMD at 32 vectors (134
// registers; left to itself the compiler took 144 + 64 and ran two).
template <int BN, int BM = 64>
__global__ __launch_bounds__(DN_NT) __attribute__((amdgpu_waves_per_eu(BM == 32 ? 3 : 2))) void k_dense(const double *__restrict__ At, int npad, VecRef vr,
                                                 const double *__restrict__ alpha, int64_t ld,
                                                 double *__restrict__ beta, int64_t N0, int64_t batch)
{
    constexpr int AW = BN + 16;            // matrix tile row stride: rows alternate LDS bank halves
    constexpr int AL = DN_BK * BN / DN_NT; // matrix values per thread per chunk
    constexpr int AR = DN_NT / BN;         // chunk rows loaded in one sweep of the workgroup
    constexpr int DN_XL = BM * DN_BK / DN_NT; // alpha values per thread per chunk
    constexpr int VG = BM / 16, TS = 4 / VG;  // vector groups; tile stride of a wave
    static_assert(BN % DN_BK == 0 && AL * DN_NT == DN_BK * BN && AR * BN == DN_NT, "dense tiling");
    static_assert(DN_XL * DN_NT == BM * DN_BK && VG * TS == 4, "dense tiling");
    __shared__ double xs[BM * DN_XW];
    __shared__ double as[DN_BK * AW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int vg = w % VG, t0 = w / VG;
    const int64_t b0 = (int64_t)blockIdx.x * BM;
    const int j0 = blockIdx.y * BN;
    const int jend = min(npad, j0 + BN);
    // alpha loader: chunk column xc, vector rows xr0 + 16 e
    const int xc = threadIdx.x % DN_BK, xr0 = threadIdx.x / DN_BK;
    int64_t lbase[DN_XL], ln[DN_XL];
#pragma unroll
    for (int e = 0; e < DN_XL; ++e) {
        const int64_t b = b0 + xr0 + (DN_NT / DN_BK) * e;
        if (b < batch) vec_of(vr, b, ld, N0, lbase[e], ln[e]);
        else lbase[e] = 0, ln[e] = -1;
    }
    // matrix loader: output column j0 + threadIdx.x % BN of chunk rows ar0 + AR e
    const int ac = (int)threadIdx.x % BN, ar0 = (int)threadIdx.x / BN;
    const int aj = j0 + ac;
    double xreg[DN_XL], areg[AL];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int e = 0; e < DN_XL; ++e) {
            const int64_t k = kc + xc;
            xreg[e] = k <= ln[e] ? alpha[lbase[e] + k] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < AL; ++e) {
            const int k = kc + ar0 + AR * e;
            // At[k][j] = 0 for j > k
            areg[e] = (aj < npad && aj <= k) ? At[(int64_t)k * npad + aj] : 0.0;
        }
    };
    constexpr int NTL = BN / 16 / TS; // output tiles per chunk and wave: t0 + TS i
    v4d acc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = v4d{0, 0, 0, 0};
    // the chunk starting at output j0 needs k >= j0 only
    fetch(j0);
    for (int kc = j0; kc < npad; kc += DN_BK) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < DN_XL; ++e) xs[(xr0 + (DN_NT / DN_BK) * e) * DN_XW + xc] = xreg[e];
#pragma unroll
        for (int e = 0; e < AL; ++e) as[(ar0 + AR * e) * AW + ac] = areg[e];
        __syncthreads();
        if (kc + DN_BK < npad) fetch(kc + DN_BK);
#pragma unroll
        for (int ks = 0; ks < DN_BK; ks += 4) {
            const int k0 = kc + ks;
            const double a = xs[(16 * vg + (lane & 15)) * DN_XW + ks + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < NTL; ++t) {
                const int jl = 16 * (t0 + TS * t);
                if (j0 + jl >= jend || k0 + 4 <= j0 + jl) continue; // outside the matrix, or all zero there
                const double bv = as[(ks + (lane >> 4)) * AW + jl + (lane & 15)];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t], 0, 0, 0);
            }
        }
    }
    int64_t sbase[4], sn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t b = b0 + 16 * vg + (lane >> 4) + 4 * i;
        if (b < batch) vec_of(vr, b, ld, N0, sbase[i], sn[i]);
        else sbase[i] = 0, sn[i] = -1;
    }
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        const int jt = j0 + 16 * (t0 + TS * t);
        if (jt >= jend) continue;
        const int64_t j = jt + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (j <= sn[i]) beta[sbase[i] + j] = acc[t][i];
    }
}

void launch_dense(const double *At, int64_t npad, const int64_t *off, const int64_t *deg,
                  const double *alpha, int64_t ld, double *beta, int64_t N, int64_t batch,
                  hipStream_t s)
{
    if (batch <= 0) return;
    const unsigned gx = (unsigned)((batch + 63) / 64);
    if ((int64_t)gx * ((npad + 255) / 256) >= 512) {
        // 32 vectors per workgroup: three workgroups per CU instead of two
        // (measured 3% faster than 64 at 65536 x degree 255)
        constexpr int BM = 32;
        dim3 grid((unsigned)((batch + BM - 1) / BM), (unsigned)((npad + 255) / 256));
        k_dense<256, BM><<<grid, DN_NT, 0, s>>>(At, (int)npad, VecRef{off, deg}, alpha, ld, beta, N, batch);
    } else {
        dim3 grid(gx, (unsigned)((npad + 63) / 64));
        k_dense<64><<<grid, DN_NT, 0, s>>>(At, (int)npad, VecRef{off, deg}, alpha, ld, beta, N, batch);
    }
}

// ---- the same product in split bfloat16 (FP32-bulk plans) ------------------------
// Every FP32 value is the exact sum of three bfloat16 parts x = h + m + l: h keeps
// the top 8 significant bits (the low half of the encoding cleared), the
// remainder x - h is exact in FP32 and has at most 16 significant bits, m keeps
// its top 8, and the last remainder (at most 8 bits) is l; |m| < 2^-7 |x| and
// |l| < 2^-14 |x|.  Of the nine partial products eight are summed on the matrix
// cores in FP32, smallest first (every bfloat16 product is exact in FP32); the
// dropped l l is below 2^-28 |a b|.  The result is an FP32-accurate product at
// the bfloat16 rate of the matrix cores.
//
// v_mfma_f32_16x16x32_bf16 lane layout (lane l, m = l & 15, g = l >> 4):
// operand a = X[m][8g .. 8g+7], operand b = Y[8g .. 8g+7][n = l & 15], result
// element i = D[4g + i][l & 15].
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
constexpr int DB_VB = 64;  // vectors per workgroup: wave w owns vectors 16w .. 16w + 15
constexpr int DB_NT = 256;
constexpr int DB_KC = 32;  // k per chunk (one matrix-core step)
static_assert(DENSE_PAD % DB_KC == 0, "dense padding");

// the three parts of 8 consecutive values, packed two per dword (element 2i in
// the low half): h, m, l
__device__ __forceinline__ void split_bf16x3(const float *f, v4u &h, v4u &m, v4u &l)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        unsigned uh[2], um[2], ul[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned u = __float_as_uint(f[2 * i + q]);
            uh[q] = u & 0xffff0000u;
            const float r1 = f[2 * i + q] - __uint_as_float(uh[q]);
            um[q] = __float_as_uint(r1) & 0xffff0000u;
            const float r2 = r1 - __uint_as_float(um[q]);
            ul[q] = __float_as_uint(r2) & 0xffff0000u;
        }
        h[i] = (uh[0] >> 16) | uh[1];
        m[i] = (um[0] >> 16) | um[1];
        l[i] = (ul[0] >> 16) | ul[1];
    }
}

// Bp[((kc * 3 + part) * npad + j) * 32 + kk] = part of At[32 kc + kk][j]: a
// lane's eight consecutive k of one column are one 16-byte load
__global__ void k_split_matrix(const double *__restrict__ At, int npad, v4u *__restrict__ Bp)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; // (j, kc, kg)
    const int nkc = npad / DB_KC;
    if (q >= (int64_t)npad * nkc * 4) return;
    const int kg = (int)(q & 3);
    const int kc = (int)((q >> 2) % nkc);
    const int j = (int)((q >> 2) / nkc);
    float f[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = (float)At[(int64_t)(DB_KC * kc + 8 * kg + i) * npad + j];
    v4u h, m, l;
    split_bf16x3(f, h, m, l);
    const int64_t base = ((int64_t)kc * 3 * npad + j) * 4 + kg; // in 16-byte units
    Bp[base] = h;
    Bp[base + (int64_t)npad * 4] = m;
    Bp[base + (int64_t)npad * 8] = l;
}

// Workgroup: 64 vectors x JB outputs (JB = 256, or 64 when there are too few
// vectors to give every CU a workgroup of 256 outputs).  Per chunk of 32 k the
// workgroup stages the matrix parts of its JB columns in LDS (coalesced 16-byte
// loads, read into registers one chunk ahead); each wave reads the alpha values
// of its own 16 vectors straight into operand registers (two chunks ahead),
// splits them, and runs 8 products per output tile of the chunk.  Compiled for
// two waves per SIMD at 256 outputs (left to itself the compiler took 256 + 64
// registers and ran one).
template <int JB>
__global__ __launch_bounds__(DB_NT) __attribute__((amdgpu_waves_per_eu(JB == 256 ? 2 : 4))) void k_dense_bf16(const v4u *__restrict__ Bp, int npad, VecRef vr,
                                                      const double *__restrict__ alpha, int64_t ld,
                                                      double *__restrict__ beta, int64_t N0, int64_t batch)
{
    constexpr int NTL = JB / 16;               // output tiles
    constexpr int BU = 3 * JB * 4;             // 16-byte units of one chunk's matrix parts
    constexpr int BL = BU / DB_NT;             // of them per thread
    static_assert(BL * DB_NT == BU, "matrix chunk loader");
    __shared__ v4u bs[BU];                     // [part][column][k group]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int64_t b0 = (int64_t)blockIdx.x * DB_VB;
    const int j0 = blockIdx.y * JB;
    const int jn = min(JB, npad - j0);          // columns of this workgroup inside the matrix
    int64_t abase, an;
    if (b0 + 16 * w + m < batch) vec_of(vr, b0 + 16 * w + m, ld, N0, abase, an);
    else abase = 0, an = -1;
    // alpha runs two chunks ahead (two register sets, the loop unrolled by two so
    // that each set keeps its registers), the matrix parts one chunk ahead: with two
    // workgroups per CU that keeps about 64 KiB of alpha reads in flight per CU
    double xa[8], xb[8];
    v4u br[BL];
    auto fetch_alpha = [&](int kc, double *xr) {
        const int64_t k0 = (int64_t)DB_KC * kc + 8 * g;
        if (k0 + 7 <= an && ((abase + k0) & 1) == 0) {
            // the lane's eight values inside the vector and 16-byte aligned: four 16-byte loads
            const double2 *p = reinterpret_cast<const double2 *>(alpha + abase + k0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double2 v = p[i];
                xr[2 * i] = v.x;
                xr[2 * i + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) xr[i] = k0 + i <= an ? alpha[abase + k0 + i] : 0.0;
        }
    };
    // columns from DB_KC (kc + 1) on are zero in chunk kc (At[k][j] = 0 for k < j) and
    // their tiles are skipped, so they are neither read nor staged
    auto fetch_matrix = [&](int kc) {
        const int jlim = min(jn, DB_KC * (kc + 1) - j0);
#pragma unroll
        for (int e = 0; e < BL; ++e) {
            const int u = (int)threadIdx.x + DB_NT * e; // (part, column, k group)
            const int p = u / (JB * 4), r = u % (JB * 4);
            br[e] = (r >> 2) < jlim ? Bp[((int64_t)(kc * 3 + p) * npad + j0) * 4 + r] : v4u{0, 0, 0, 0};
        }
    };
    v4f acc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = v4f{0, 0, 0, 0};
    const int nkc = npad / DB_KC;
    // one chunk: stage the matrix parts, split the chunk's alpha (xr) into bfloat16
    // parts, refill xr with the chunk two ahead, and accumulate every tile the
    // chunk reaches
    auto chunk = [&](int kc, double *xr) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < BL; ++e) bs[threadIdx.x + DB_NT * e] = br[e];
        float f[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = (float)xr[i];
        __syncthreads();
        if (kc + 1 < nkc) fetch_matrix(kc + 1);
        if (kc + 2 < nkc) fetch_alpha(kc + 2, xr);
        v4u xh, xm, xl;
        split_bf16x3(f, xh, xm, xl);
        const v8bf ah = __builtin_bit_cast(v8bf, xh), am = __builtin_bit_cast(v8bf, xm),
                   al = __builtin_bit_cast(v8bf, xl);
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
            const int jl = 16 * t;
            // outside the matrix, or every k of the chunk below the tile
            if (jl >= jn || DB_KC * kc + DB_KC <= j0 + jl) continue;
            const v8bf bh = __builtin_bit_cast(v8bf, bs[(0 * JB + jl + m) * 4 + g]);
            const v8bf bm = __builtin_bit_cast(v8bf, bs[(1 * JB + jl + m) * 4 + g]);
            const v8bf bl = __builtin_bit_cast(v8bf, bs[(2 * JB + jl + m) * 4 + g]);
            v4f c = acc[t];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bm, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, c, 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
        }
    };
    // chunks of k below the first output are zero (At[k][j] = 0 for k < j)
    const int kc0 = j0 / DB_KC;
    fetch_alpha(kc0, xa);
    fetch_matrix(kc0);
    if (kc0 + 1 < nkc) fetch_alpha(kc0 + 1, xb);
    for (int kc = kc0; kc < nkc; kc += 2) {
        chunk(kc, xa);
        if (kc + 1 < nkc) chunk(kc + 1, xb);
    }
    int64_t sbase[4], sn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t b = b0 + 16 * w + 4 * g + r;
        if (b < batch) vec_of(vr, b, ld, N0, sbase[r], sn[r]);
        else sbase[r] = 0, sn[r] = -1;
    }
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        if (16 * t >= jn) continue;
        const int64_t j = j0 + 16 * t + m;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (j <= sn[r]) beta[sbase[r] + j] = (double)acc[t][r];
    }
}

int64_t dense_bf16_elems(int64_t npad) { return 3 * npad * npad; }

void launch_split_matrix(const double *At, int64_t npad, void *Bp, hipStream_t s)
{
    const int64_t n = npad * (npad / DB_KC) * 4;
    k_split_matrix<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(At, (int)npad, (v4u *)Bp);
}

void launch_dense_bf16(const void *Bp, int64_t npad, const int64_t *off, const int64_t *deg,
                       const double *alpha, int64_t ld, double *beta, int64_t N, int64_t batch,
                       hipStream_t s)
{
    if (batch <= 0) return;
    const unsigned gx = (unsigned)((batch + DB_VB - 1) / DB_VB);
    if ((int64_t)gx * ((npad + 255) / 256) >= 512) {
        dim3 grid(gx, (unsigned)((npad + 255) / 256));
        k_dense_bf16<256><<<grid, DB_NT, 0, s>>>((const v4u *)Bp, (int)npad, VecRef{off, deg}, alpha, ld,
                                                 beta, N, batch);
    } else {
        dim3 grid(gx, (unsigned)((npad + 63) / 64));
        k_dense_bf16<64><<<grid, DB_NT, 0, s>>>((const v4u *)Bp, (int)npad, VecRef{off, deg}, alpha, ld,
                                                beta, N, batch);
    }
}

// ============================================================================
// a5: sums of diagonally scaled Toeplitz products, eq. (Cdecomposition)
// ============================================================================

// Largest radix of the register FFTs.  Radix 8 keeps 8 values per thread, so a
// workgroup of M*NB/8 threads holds the transform: twice the waves of radix 16
// at the same LDS footprint, which is what hides HBM latency in these passes.
// The single-workgroup path also has radix 16 (half the threads, one LDS
// exchange fewer at 4096 points); the autotuner picks per plan.
constexpr int RMAX = 8;
template <int M, int NB, int R = RMAX>
constexpr int nthreads() { return fft_threads(M, NB, R); }

// One workgroup per (slot group, vector): for each slot s of the group
//   z = l~_s o X (zero-padded to L) -> FFT -> . that -> IFFT -> acc += l~_s o y
// with `that` = FFT(symbol)/L.  The accumulator stays in registers, in the
// forward-input layout that the inverse transform returns to.
template <typename T, int L, int R, bool AIN>
__global__ __launch_bounds__((nthreads<L, 1, R>())) void k_toep_lds(
    const cpx<T> *__restrict__ X, int64_t nc, int64_t n, const cpx<T> *__restrict__ ell, int S,
    int spg, const cpx<T> *__restrict__ that, const cpx<T> *__restrict__ tw, cpx<T> *__restrict__ W,
    int64_t batch, AlphaIn ain)
{
    // twiddle reads a stage ahead: one vector of degree 2048 (26 workgroups,
    // latency-bound) measured 14.0 -> 12.8 us per conversion
    using F = RegFFT<T, L, 1, nthreads<L, 1, R>(), R, true>;
    constexpr int E = F::E;
    // Only positions below n <= L/2 + 1 are loaded or kept.  In the forward
    // input layout (= the inverse's output layout) slot e holds position
    // w + r L/RF (r = e mod RF, w < L/RF): slots with r > RF/2 are always zero
    // on input and discarded on output; slot RF/2 of thread 0 holds position
    // L/2, the only one of them that can be below n.
    constexpr int RF = F::R_FIRST, RH = RF / 2;
    static_assert(RF >= 2, "first radix");
    constexpr int EH = (E / RF) * RH;
    __shared__ cpx<T> lds[F::LDS];
    const int g = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int s0 = g * spg;
    const int s1 = min(S, s0 + spg);
    cpx<T> acc[EH], accm{0, 0}, v[E];
#pragma unroll
    for (int h = 0; h < EH; ++h) acc[h] = cpx<T>{0, 0};
    int pmid, cmid;
    F::in_pos(RH, pmid, cmid);
    // In double precision the packed input, the symbol and l~_s are read again
    // where they are used (cache hits) rather than kept live across the
    // transforms: opaque pointers stop the loads from being hoisted out of the
    // slot loop (fewer registers; measured faster for FP64; in FP32 needed at
    // 8192 points, where the hoisted values spill).
    auto opq = [](const cpx<T> *q) { return sizeof(T) == 8 || L >= 8192 ? opaque_ptr(q) : q; };
    // input lanes from the packed X, or (AIN) formed from the vector itself
    int64_t abase = 0, aN = -1;
    if constexpr (AIN) vec_of(VecRef{ain.off, ain.deg}, b, ain.ld, ain.N0, abase, aN);
    for (int s = s0; s < s1; ++s) {
        const cpx<T> *es = opq(ell + (int64_t)s * nc);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int pos, c;
            F::in_pos(e, pos, c);
            if (e % RF <= RH && pos < n) {
                if constexpr (AIN) v[e] = cdiag(es[pos], x_lane<T>(ain.k, opaque_ptr(ain.alpha + abase), aN, pos));
                else v[e] = cdiag(es[pos], opq(X + b * nc)[pos]);
            } else {
                v[e] = cpx<T>{0, 0};
            }
        }
        F::forward(v, lds, tw);
        const cpx<T> *ts = opq(that);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int pos, c;
            F::out_pos(e, pos, c);
            v[e] = cmul(v[e], ts[pos]);
        }
        F::inverse(v, lds, tw);
        es = opq(es);
#pragma unroll
        for (int h = 0; h < EH; ++h) {
            const int e = (h / RH) * RF + h % RH;
            int pos, c;
            F::in_pos(e, pos, c);
            if (pos < n) acc[h] = cadd(acc[h], cdiag(es[pos], v[e]));
        }
        if (pmid < n) accm = cadd(accm, cdiag(es[pmid], v[RH]));
    }
    cpx<T> *Wg = W + ((int64_t)g * batch + b) * nc;
#pragma unroll
    for (int h = 0; h < EH; ++h) {
        int pos, c;
        F::in_pos((h / RH) * RF + h % RH, pos, c);
        if (pos < n) Wg[pos] = acc[h];
    }
    if (pmid < n) Wg[pmid] = accm;
}

template <typename T, int L>
__global__ __launch_bounds__((nthreads<L, 1>())) void k_fft_lds(const cpx<T> *in, cpx<T> *out,
                                                                  const cpx<T> *tw, T scale)
{
    using F = RegFFT<T, L, 1, nthreads<L, 1>(), RMAX>;
    __shared__ cpx<T> lds[F::LDS];
    cpx<T> v[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        int pos, c;
        F::in_pos(e, pos, c);
        v[e] = in[pos];
    }
    F::forward(v, lds, tw);
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        int pos, c;
        F::out_pos(e, pos, c);
        out[pos] = cpx<T>{v[e].x * scale, v[e].y * scale};
    }
}

template <typename T, int L, int R>
static void run_toep_lds(const void *X, int64_t nc, int64_t n, const void *ell, int S, int spg, int G,
                         const void *that, const void *tw, void *W, int64_t batch, hipStream_t s,
                         const AlphaIn &ain)
{
    dim3 grid((unsigned)G, (unsigned)batch);
    if (ain.alpha)
        k_toep_lds<T, L, R, true><<<grid, nthreads<L, 1, R>(), 0, s>>>(
            (const cpx<T> *)X, nc, n, (const cpx<T> *)ell, S, spg, (const cpx<T> *)that, (const cpx<T> *)tw,
            (cpx<T> *)W, batch, ain);
    else
        k_toep_lds<T, L, R, false><<<grid, nthreads<L, 1, R>(), 0, s>>>(
            (const cpx<T> *)X, nc, n, (const cpx<T> *)ell, S, spg, (const cpx<T> *)that, (const cpx<T> *)tw,
            (cpx<T> *)W, batch, ain);
}

template <typename T, int L>
static void run_toep_lds_r(int radix, const void *X, int64_t nc, int64_t n, const void *ell, int S, int spg,
                           int G, const void *that, const void *tw, void *W, int64_t batch, hipStream_t s,
                           const AlphaIn &ain)
{
    if (radix == 16) run_toep_lds<T, L, 16>(X, nc, n, ell, S, spg, G, that, tw, W, batch, s, ain);
    else run_toep_lds<T, L, 8>(X, nc, n, ell, S, spg, G, that, tw, W, batch, s, ain);
}

template <typename T>
bool launch_toep_lds(int64_t L, int radix, const void *X, int64_t nc, int64_t n, const void *ell, int S,
                     int spg, int G, const void *that, const void *tw, void *W, int64_t batch,
                     hipStream_t s, const AlphaIn *ainp)
{
    if (n > L / 2 + 1 || n > nc) return false; // the kernel loads and keeps positions below L/2 + 1 only
    if (radix != 8 && radix != 16) return false;
    if (!X && !(ainp && ainp->alpha)) return false;
    AlphaIn ain{};
    if (ainp) ain = *ainp;
    switch (L) {
#define THX_CASE(LL) case LL: run_toep_lds_r<T, LL>(radix, X, nc, n, ell, S, spg, G, that, tw, W, batch, s, ain); return true;
        THX_CASE(64) THX_CASE(128) THX_CASE(256) THX_CASE(512) THX_CASE(1024) THX_CASE(2048)
        THX_CASE(4096)
#undef THX_CASE
    case 8192:
        if constexpr (sizeof(T) == 4) {
            run_toep_lds_r<T, 8192>(radix, X, nc, n, ell, S, spg, G, that, tw, W, batch, s, ain);
            return true;
        }
        return false;
    default: return false;
    }
}
template bool launch_toep_lds<double>(int64_t, int, const void *, int64_t, int64_t, const void *, int, int, int, const void *, const void *, void *, int64_t, hipStream_t, const AlphaIn *);
template bool launch_toep_lds<float>(int64_t, int, const void *, int64_t, int64_t, const void *, int, int, int, const void *, const void *, void *, int64_t, hipStream_t, const AlphaIn *);

template <typename T>
bool launch_fft_lds(int64_t L, const void *in, void *out, const void *tw, double scale, hipStream_t s)
{
    switch (L) {
#define THX_CASE(LL) case LL: k_fft_lds<T, LL><<<1, nthreads<LL, 1>(), 0, s>>>((const cpx<T> *)in, (cpx<T> *)out, (const cpx<T> *)tw, (T)scale); return true;
        THX_CASE(64) THX_CASE(128) THX_CASE(256) THX_CASE(512) THX_CASE(1024) THX_CASE(2048)
        THX_CASE(4096)
#undef THX_CASE
    case 8192:
        if constexpr (sizeof(T) == 4) {
            k_fft_lds<T, 8192><<<1, nthreads<8192, 1>(), 0, s>>>((const cpx<T> *)in, (cpx<T> *)out,
                                                                  (const cpx<T> *)tw, (T)scale);
            return true;
        }
        return false;
    default: return false;
    }
}
template bool launch_fft_lds<double>(int64_t, const void *, void *, const void *, double, hipStream_t);
template bool launch_fft_lds<float>(int64_t, const void *, void *, const void *, double, hipStream_t);

// ---------------------------------------------------------------------------
// Three-pass (four-step) FFT for L = L1 * L2 > one workgroup's LDS.
// Index a = a1 + L1 a2 (a1 < L1 fast), frequency k = k2 + L2 k1.
//   P1: column DFTs over a2 (length L2) for TC adjacent columns, twiddle
//       w_L^{a1 k2}, result at position a1 + L1 k2;
//   P2: each row k2 (contiguous, length L1): DFT over a1 gives Z[k2 + L2 k1];
//       multiply by the symbol stored in the same permuted order, inverse DFT,
//       conjugate twiddle w_L^{-a1 k2};
//   P3: inverse column DFTs over k2 give y[a1 + L1 a2] in natural order, which
//       is scaled by l~_s and summed over the slots of the group.
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Map the 1-D block index b to (item, rep) so that the `reps` blocks that share
// `item`'s data (a symbol row, an input tile) run back to back on one XCD.
// Requires items % 8 == 0; otherwise reps of an item are simply consecutive.
__device__ __forceinline__ void xcd_map(int b, int items, int reps, int &item, int &rep)
{
    if (items & 7) {
        item = b / reps;
        rep = b % reps;
        return;
    }
    const int x = b & 7, m = b >> 3;
    item = x + 8 * (m / reps);
    rep = m % reps;
}

// Points per column-pass workgroup.  FP64: 4096 (two workgroups per CU), or
// 8192 for columns of 512 and more, so that a tile still spans 16 adjacent
// columns (256-byte segments; one 1024-thread workgroup per CU in 136 KiB of
// LDS) -- measured 2% faster per execution at L2 = 512, while 32-column tiles
// at L2 = 256 measured 8% slower than 16.  FP32: 8192 (16384 spilled), except
// 4096 for columns of 128 and 256 (tiles of 32 and 16 columns, four workgroups
// per CU instead of two): both column passes 9-10% faster at L2 = 256.
template <typename T, int L2>
constexpr int mp_tile()
{
    return sizeof(T) == 4 ? ((L2 == 128 || L2 == 256) ? 4096 : 8192) : (L2 >= 512 ? 8192 : 4096);
}
constexpr int64_t pow2_floor(int64_t x) { return x < 2 ? 1 : 2 * pow2_floor(x / 2); }
// Columns of 3 * 2^m and 5 * 2^m (lengths L = 3 * 2^k and 5 * 2^k, which pad
// mixed batches less) take radix-4 stages and one radix-3 or radix-5 stage with
// 12 or 20 values per thread (6 for columns of 6, 10 for columns of 10), so that
// every radix divides the per-thread count; their tiles are the largest
// power-of-two number of columns that fits.
template <int L2> constexpr bool col_mixed() { return L2 % 3 == 0 || L2 % 5 == 0; }
template <int L2> constexpr int col_rmax() { return col_mixed<L2>() ? 4 : RMAX; }
template <int L2> constexpr int col_e() { return L2 % 5 == 0 ? (L2 == 10 ? 10 : 20) : (L2 == 6 ? 6 : 12); }
template <typename T, int L2>
constexpr int mp_tc()
{
    return (int)std::min<int64_t>(64, pow2_floor(mp_tile<T, L2>() / L2));
}
template <typename T, int L2>
constexpr int mp_nt()
{
    if constexpr (col_mixed<L2>()) return mp_tc<T, L2>() * L2 / col_e<L2>();
    else return nthreads<L2, mp_tc<T, L2>()>();
}
// PREF (twiddle reads a stage ahead) only for columns of 2^m: the mixed-radix
// columns' 12 or 20 values per thread leave no registers for them
template <typename T, int L2, bool PREF = false>
using ColFFT = RegFFT<T, L2, mp_tc<T, L2>(), mp_nt<T, L2>(), col_rmax<L2>(), PREF && !col_mixed<L2>()>;

// columns the three-pass kernels are built for: 2^m (2 ... 1024), 3 * 2^m (6 ... 768)
// or 5 * 2^m (10 ... 640; a column of 5 would start its inverse with an odd radix,
// which the inverse pass's split of kept outputs at L2/2 does not handle)
static bool column_length_ok(int64_t L2)
{
    if (L2 < 2) return false;
    const int64_t q = L2 % 3 == 0 ? 3 : (L2 % 5 == 0 ? 5 : 1), P = L2 / q;
    if ((P & (P - 1)) != 0) return false;
    if (q == 3) return L2 >= 6 && L2 <= 768;
    if (q == 5) return L2 >= 10 && L2 <= 640;
    return L2 <= 1024;
}

bool multipass_ok(int64_t L, int64_t L1)
{
    return L1 > 0 && L % L1 == 0 && column_length_ok(L / L1);
}

template <typename T>
MultiPassGeom multipass_geom(int64_t L, int64_t row)
{
    MultiPassGeom g;
    g.L = L;
    const bool xl = mp_row_xl<T>() > 0 && row == mp_row_xl<T>() && L % row == 0 &&
                    (L / row == 256 || L / row == 512);
    const bool ok = xl || ((row == mp_row_short<T>() || row == mp_row_long<T>()) && L % row == 0 &&
                           column_length_ok(L / row));
    if (!ok) row = L / mp_row_short<T>() <= 512 ? mp_row_short<T>() : mp_row_long<T>();
    g.L1 = row;
    g.L2 = L / g.L1;
    const int64_t tile = sizeof(T) == 4 ? ((g.L2 == 128 || g.L2 == 256) ? 4096 : 8192)
                                        : (g.L2 >= 512 ? 8192 : 4096); // mp_tile<T, L2>
    g.TC = std::min<int64_t>(64, pow2_floor(tile / g.L2));                    // mp_tc<T, L2>
    return g;
}
template MultiPassGeom multipass_geom<double>(int64_t, int64_t);
template MultiPassGeom multipass_geom<float>(int64_t, int64_t);

// w_L^e for 0 <= e < L = L1 L2, from twA[e] = w_L^e (e < L1) and twL2[i] = w_L^{i L1}
template <typename T, int L1>
__device__ __forceinline__ cpx<T> tw_L(const cpx<T> *__restrict__ twA, const cpx<T> *__restrict__ twL2, int e)
{
    return cmul(twA[e & (L1 - 1)], twL2[e >> ilog2(L1)]);
}

// A workgroup transforms one column tile of one vector, for one slot (SG =
// false, spb = 1) or for `spb` consecutive slots (SG = true: the packed-input
// tile stays in registers across them; a separate instantiation, because the
// values it keeps live would make the single-slot kernel spill at 1024 threads).
template <typename T, int L1, int L2, bool SG>
__global__ __launch_bounds__((mp_nt<T, L2>())) void k_mp_p1(
    const cpx<T> *__restrict__ X, int64_t nc, int64_t n, const cpx<T> *__restrict__ ell, int slot0,
    int nslots, int spb, const cpx<T> *__restrict__ src, cpx<T> *__restrict__ U, int64_t batch,
    const cpx<T> *__restrict__ twL2, const cpx<T> *__restrict__ twA, AlphaIn ain)
{
    constexpr int TC = mp_tc<T, L2>();
    constexpr int NT = mp_nt<T, L2>();
    // twiddle reads a stage ahead, except with slot groups (their registers
    // hold the tile's input across slots)
    using F = ColFFT<T, L2, !SG>;
    constexpr int64_t L = (int64_t)L1 * L2;
    __shared__ cpx<T> lds[F::LDS];
    constexpr int tiles = L1 / TC;
    constexpr int RF = F::R_FIRST;
    // tiles fastest: consecutive blocks write adjacent columns of the same rows
    const int a1_0 = (int)(blockIdx.x % tiles) * TC;
    const int nsg = (nslots + spb - 1) / spb;
    const int sg = (int)((blockIdx.x / tiles) % nsg);
    const int64_t b = blockIdx.x / (tiles * nsg);
    const cpx<T> *Xb = X ? X + b * nc : nullptr;
    // lanes formed from the vector itself when no packed X is given (with slot
    // groups once per workgroup, before the slot loop)
    int64_t abase = 0, aN = -1;
    if (ain.alpha) vec_of(VecRef{ain.off, ain.deg}, b, ain.ld, ain.N0, abase, aN);
    auto xin = [&](int64_t a) -> cpx<T> {
        return ain.alpha ? x_lane<T>(ain.k, ain.alpha + abase, aN, a) : Xb[a];
    };
    // slots e with e mod RF > RF/2 hold positions above L/2: zero padding
    auto live = [&](int e, int64_t a) { return e % RF <= RF / 2 && a < n; };
    auto transform_store = [&](cpx<T> *v, int sl) {
        F::forward(v, lds, twL2);
        cpx<T> *Ub = U + ((int64_t)sl * batch + b) * L;
        // Twiddle w_L^{a1 k2}.  The thread's column a1 is the same in all its
        // butterfly groups p and its rows are k2 = j_p + q L2/RL, so the factor is
        // w_L^{a1 j_p} (one table pair per group) times the q-th power of
        // w_L^{a1 L2/RL} (powers of two from the tables, the rest as products).
        constexpr int RL = F::R_LAST, PG = F::E / RL;
        static_assert(NT % TC == 0, "column of a thread fixed across groups");
        const int a1 = a1_0 + (int)threadIdx.x % TC;
        cpx<T> st[RL];
        st[0] = cpx<T>{1, 0};
#pragma unroll
        for (int q = 1; q < RL; ++q) {
            if ((q & (q - 1)) == 0) st[q] = tw_L<T, L1>(twA, twL2, a1 * q * (L2 / RL));
            else st[q] = cmul(st[q & (q - 1)], st[q & -q]);
        }
#pragma unroll
        for (int p = 0; p < PG; ++p) {
            const int j = ((int)threadIdx.x + NT * p) / TC;
            const cpx<T> bp = tw_L<T, L1>(twA, twL2, a1 * j);
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                const int k2 = j + q * (L2 / RL);
                const cpx<T> t = q == 0 ? bp : cmul(bp, st[q]);
                st_stream(Ub + a1 + (int64_t)L1 * k2, cmul(v[p * RL + q], t));
            }
        }
    };
    if constexpr (!SG) {
        const int sl = sg;
        const cpx<T> *es = ell ? ell + (int64_t)(slot0 + sl) * nc : nullptr;
        cpx<T> v[F::E];
#pragma unroll
        for (int e = 0; e < F::E; ++e) {
            int a2, c;
            F::in_pos(e, a2, c);
            const int64_t a = a1_0 + c + (int64_t)L1 * a2;
            if (es) v[e] = live(e, a) ? cdiag(es[a], xin(a)) : cpx<T>{0, 0};
            else v[e] = src[a];
        }
        transform_store(v, sl);
    } else {
        const int s0 = sg * spb, s1 = min(nslots, s0 + spb);
        cpx<T> xv[F::E];
#pragma unroll
        for (int e = 0; e < F::E; ++e) {
            int a2, c;
            F::in_pos(e, a2, c);
            const int64_t a = a1_0 + c + (int64_t)L1 * a2;
            xv[e] = live(e, a) ? xin(a) : cpx<T>{0, 0};
        }
        // the next slot's l~ tile is loaded while this slot is transformed
        cpx<T> ev[F::E];
        auto load_ell = [&](int sl) {
            const cpx<T> *es = ell + (int64_t)(slot0 + sl) * nc;
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
                int a2, c;
                F::in_pos(e, a2, c);
                const int64_t a = a1_0 + c + (int64_t)L1 * a2;
                ev[e] = live(e, a) ? es[a] : cpx<T>{0, 0};
            }
        };
        if (s0 < s1) load_ell(s0);
        for (int sl = s0; sl < s1; ++sl) {
            cpx<T> v[F::E];
#pragma unroll
            for (int e = 0; e < F::E; ++e) v[e] = cdiag(ev[e], xv[e]);
            if (sl + 1 < s1) load_ell(sl + 1);
            transform_store(v, sl);
            __syncthreads(); // the next slot's transform reuses the LDS
        }
    }
}

// the row pass keeps radix 16: two LDS exchanges per transform instead of three
// (radix 8 with twice the waves per row measured slower)
constexpr int RMAX_ROW = 16;
template <typename T, int L1>
constexpr int p2_threads() { return fft_threads(L1, 1, RMAX_ROW); }

// Row k2 of the row pass, from the forward input layout in registers: DFT,
// times the permuted symbol row, inverse DFT, conjugate twiddle, stored to `row`
// (the same steps as the tail of k_mp_p2, for the fused pass).
template <typename T, int L1>
__device__ __forceinline__ void p2_row(cpx<T> *v, cpx<T> *lds, int k2, cpx<T> *__restrict__ row,
                                       const cpx<T> *__restrict__ tp, const cpx<T> *__restrict__ twL1,
                                       const cpx<T> *__restrict__ twA, const cpx<T> *__restrict__ twL2)
{
    constexpr int NT = p2_threads<T, L1>();
    using F = RegFFT<T, L1, 1, NT, RMAX_ROW, sizeof(T) == 8>;
    F::forward(v, lds, twL1);
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        int k1, c;
        F::out_pos(e, k1, c);
        v[e] = cmul(v[e], tp[k1]);
    }
    F::inverse(v, lds, twL1);
    // Conjugate twiddle w_L^{-a1 k2} with a1 = j_p + r L1/RF (j_p = threadIdx.x
    // + NT p): a per-thread factor w_L^{j_p k2} times the workgroup-uniform
    // w_L^{r k2 L1/RF}, so only one table pair per group is gathered.
    constexpr int RF = F::R_FIRST, PG = F::E / RF;
    cpx<T> bp[PG];
#pragma unroll
    for (int p = 0; p < PG; ++p) bp[p] = tw_L<T, L1>(twA, twL2, ((int)threadIdx.x + NT * p) * k2);
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        const cpx<T> sr = tw_L<T, L1>(twA, twL2, r * (L1 / RF) * k2);
#pragma unroll
        for (int p = 0; p < PG; ++p) {
            const int a1 = (int)threadIdx.x + NT * p + r * (L1 / RF);
            const cpx<T> t = r == 0 ? bp[p] : cmul(bp[p], sr);
            st_stream(row + a1, cmulc(v[p * RF + r], t));
        }
    }
}

template <typename T, int L1>
__global__ __launch_bounds__((p2_threads<T, L1>())) void k_mp_p2(cpx<T> *U, int L2, int nsb,
                                                                const cpx<T> *__restrict__ that_perm,
                                                                const cpx<T> *__restrict__ twL1,
                                                                const cpx<T> *__restrict__ twA,
                                                                const cpx<T> *__restrict__ twL2, int full,
                                                                cpx<T> *__restrict__ out, T scale)
{
    constexpr int NT = p2_threads<T, L1>();
    // twiddles read a stage ahead (in single precision this needs the
    // registers freed by the epilogue's twiddles in LDS: with those formed on
    // every lane it cost a wave per SIMD, rows of 8192 0.48 -> 0.65 ms)
    using F = RegFFT<T, L1, 1, NT, RMAX_ROW, true>;
    constexpr int RF = F::R_FIRST, PG = F::E / RF;
    // the exchange area, then the RF workgroup-uniform epilogue twiddles
    __shared__ cpx<T> lds[F::LDS + RF];
    int k2, sb;
    xcd_map(blockIdx.x, L2, nsb, k2, sb);
    // w_L^{r k2 L1/RF}, formed once per workgroup instead of on every lane (the
    // transforms' barriers order these writes before the epilogue's reads)
    if (full && (int)threadIdx.x < RF) lds[F::LDS + threadIdx.x] = tw_L<T, L1>(twA, twL2, (int)threadIdx.x * (L1 / RF) * k2);
    const int64_t L = (int64_t)L1 * L2;
    cpx<T> *row = U + (int64_t)sb * L + (int64_t)k2 * L1;
    cpx<T> v[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        int pos, c;
        F::in_pos(e, pos, c);
        v[e] = ld_stream(row + pos);
    }
    F::forward(v, lds, twL1);
    if (!full) {
#pragma unroll
        for (int e = 0; e < F::E; ++e) {
            int k1, c;
            F::out_pos(e, k1, c);
            out[(int64_t)k2 * L1 + k1] = cpx<T>{v[e].x * scale, v[e].y * scale};
        }
        return;
    }
    const cpx<T> *tp = that_perm + (int64_t)k2 * L1;
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        int k1, c;
        F::out_pos(e, k1, c);
        v[e] = cmul(v[e], tp[k1]);
    }
    F::inverse(v, lds, twL1);
    // Conjugate twiddle w_L^{-a1 k2} with a1 = j_p + r L1/RF (j_p = threadIdx.x
    // + NT p): a per-thread factor w_L^{j_p k2} times the workgroup-uniform
    // w_L^{r k2 L1/RF} (from LDS), so only one table pair per group is gathered.
    cpx<T> bp[PG];
#pragma unroll
    for (int p = 0; p < PG; ++p) bp[p] = tw_L<T, L1>(twA, twL2, ((int)threadIdx.x + NT * p) * k2);
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        const cpx<T> sr = lds[F::LDS + r];
#pragma unroll
        for (int p = 0; p < PG; ++p) {
            const int a1 = (int)threadIdx.x + NT * p + r * (L1 / RF);
            const cpx<T> t = r == 0 ? bp[p] : cmul(bp[p], sr);
            st_stream(row + a1, cmulc(v[p * RF + r], t));
        }
    }
}

// Row pass with the forward column pass fused in, for short columns (L2 = 2 or
// 4).  The input l~_s o X is zero at positions a >= n (<= L/2 + 1), i.e. at
// column entries a2 > L2/2, and at a2 = L2/2 except a = L/2, so the column DFT
// for row k2 is a direct sum of L2/2 terms (+ the one at L/2):
//   Y[a1, k2] = w_L^{a1 k2} sum_{a2 < L2/2} x[a1 + L1 a2] w_{L2}^{a2 k2}
//               (+ (-1)^k2 x[L/2] at a1 = 0).
// The row's workgroup reads those inputs itself (the L2 rows of one slot and
// vector run back to back on one XCD, so the reads after the first hit its L2)
// and no intermediate array is written or read before the row transforms.
// Every row reads all L2/2 nonzero column entries, so the reads grow with L2:
// measured faster than the two passes it replaces at L2 = 2 (0.69 against
// 0.93 ms for 339 vectors of degree 8182, FP64), about even at 4, and 40%
// slower at 8, which is therefore not built.
template <typename T, int L1, int L2>
__global__ __launch_bounds__((p2_threads<T, L1>())) void k_mp_p2f(
    const cpx<T> *__restrict__ X, int64_t nc, int64_t n, const cpx<T> *__restrict__ ell, int slot0,
    int nslots, cpx<T> *__restrict__ U, int64_t batch, const cpx<T> *__restrict__ that_perm,
    const cpx<T> *__restrict__ twL1, const cpx<T> *__restrict__ twA, const cpx<T> *__restrict__ twL2)
{
    static_assert(L2 == 2 || L2 == 4, "short columns only");
    constexpr int NT = p2_threads<T, L1>();
    using F = RegFFT<T, L1, 1, NT, RMAX_ROW>;
    constexpr int RF = F::R_FIRST, PG = F::E / RF;
    constexpr int64_t L = (int64_t)L1 * L2;
    __shared__ cpx<T> lds[F::LDS];
    // (slot, vector) items padded to a multiple of 8 so that the L2 rows of an
    // item share an XCD: block = xcd + 8 m, item = xcd + 8 (m / L2), row = m % L2
    const int xcd = (int)(blockIdx.x & 7), m = (int)(blockIdx.x >> 3);
    const int64_t item = xcd + 8 * (int64_t)(m / L2);
    const int k2 = m % L2;
    const int64_t nsb = (int64_t)nslots * batch;
    if (item >= nsb) return;
    const int sl = (int)(item / batch);
    const int64_t b = item % batch;
    const cpx<T> *es = ell + (int64_t)(slot0 + sl) * nc;
    const cpx<T> *Xb = X + b * nc;
    cpx<T> wk[L2 / 2];
#pragma unroll
    for (int a2 = 0; a2 < L2 / 2; ++a2) wk[a2] = twL2[(a2 * k2) & (L2 - 1)];
    cpx<T> v[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) v[e] = cpx<T>{0, 0};
#pragma unroll
    for (int a2 = 0; a2 < L2 / 2; ++a2) {
#pragma unroll
        for (int e = 0; e < F::E; ++e) {
            int a1, c;
            F::in_pos(e, a1, c);
            const int64_t a = a1 + (int64_t)L1 * a2;
            if (a < n) {
                const cpx<T> x = cdiag(es[a], Xb[a]);
                v[e] = a2 == 0 ? x : cadd(v[e], cmul(x, wk[a2]));
            }
        }
    }
    // the input at a = L/2 (column entry L2/2 of column 0: slot 0 of thread 0)
    if (threadIdx.x == 0 && L / 2 < n) {
        const cpx<T> x = cdiag(es[L / 2], Xb[L / 2]);
        v[0] = (k2 & 1) ? csub(v[0], x) : cadd(v[0], x);
    }
    // twiddle w_L^{a1 k2}, a1 = j_p + r L1/RF, factored as in the epilogue
#pragma unroll
    for (int p = 0; p < PG; ++p) {
        const cpx<T> bp = tw_L<T, L1>(twA, twL2, ((int)threadIdx.x + NT * p) * k2);
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            const cpx<T> t = r == 0 ? bp : cmul(bp, tw_L<T, L1>(twA, twL2, r * (L1 / RF) * k2));
            v[p * RF + r] = cmul(v[p * RF + r], t);
        }
    }
    cpx<T> *row = U + ((int64_t)sl * batch + b) * L + (int64_t)k2 * L1;
    p2_row<T, L1>(v, lds, k2, row, that_perm + (int64_t)k2 * L1, twL1, twA, twL2);
}

// at least four waves per SIMD for the inverse column pass, two for columns of
// 5 * 2^m, whose 20 values per thread and 10 accumulators do not fit in 128
// registers (they spill there)
template <int L2> constexpr int p3_waves() { return L2 % 5 == 0 ? 2 : 4; }

template <typename T, int L1, int L2>
__global__ __launch_bounds__((mp_nt<T, L2>())) __attribute__((amdgpu_waves_per_eu(p3_waves<L2>()))) void k_mp_p3(
    const cpx<T> *__restrict__ U, int64_t nc, int64_t n, const cpx<T> *__restrict__ ell, int slot0,
    int nslots, int spg, cpx<T> *__restrict__ W, int gofs, int64_t batch,
    const cpx<T> *__restrict__ twL2)
{
    constexpr int TC = mp_tc<T, L2>();
    // twiddle reads a stage ahead in double precision; in single precision
    // the next slot's tile is read ahead instead (both together measured
    // slower at columns of 512)
    using F = ColFFT<T, L2, sizeof(T) == 8>;
    constexpr int E = F::E;
    // Outputs kept: positions a < n <= L/2 + 1 of each sequence.  In the
    // inverse's output layout, register slot e holds column position
    // j + r L2/RF (r = e mod RF, j < L2/RF), so the slots with r < RF/2 cover
    // positions below L2/2 and only those are accumulated; the single output
    // at a = L/2 (column position L2/2 of column 0: slot RF/2 of thread 0 in
    // workgroup 0) has an accumulator of its own.
    constexpr int RF = F::R_FIRST, RH = RF / 2;
    static_assert(RF >= 2, "first radix");
    constexpr int EH = (E / RF) * RH;
    // l~_s is read with the tile (one memory round trip per slot) in single
    // precision, and in double precision for columns of 512 (measured faster
    // there; slower at 256, and it spills at 16, 32, 128 and 1024).
    constexpr bool EARLY = sizeof(T) == 4 || L2 == 512;
    __shared__ cpx<T> lds[F::LDS];
    const int a1_0 = blockIdx.x * TC;
    const int g = blockIdx.y;
    const int64_t b = blockIdx.z;
    auto kept_pos = [&](int h) {
        int a2, c;
        F::in_pos((h / RH) * RF + h % RH, a2, c);
        return a1_0 + c + (int64_t)L1 * a2;
    };
    const int64_t amid = (int64_t)L1 * (L2 / 2) + (blockIdx.x == 0 && threadIdx.x == 0 ? 0 : n);
    cpx<T> acc[EH], accm{0, 0}, v[E];
#pragma unroll
    for (int h = 0; h < EH; ++h) acc[h] = cpx<T>{0, 0};
    const int s0 = g * spg, s1 = min(nslots, (g + 1) * spg);
    auto load_tile = [&](int sl, cpx<T> *dst) {
        const cpx<T> *Ub = U + ((int64_t)sl * batch + b) * L1 * L2;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int k2, c;
            F::out_pos(e, k2, c);
            dst[e] = ld_stream(Ub + a1_0 + c + (int64_t)L1 * k2);
        }
    };
    // In single precision a tile carries half the bytes per value, so the
    // next slot's tile is loaded while this slot is transformed, which keeps
    // as many bytes in flight per wave as the double-precision pass has (in
    // double precision, and for columns of 3 * 2^m, the second tile does not
    // fit in 128 registers).
    constexpr bool PF = sizeof(T) == 4 && L2 % 3 != 0;
    cpx<T> vn[PF ? E : 1];
    if constexpr (PF)
        if (s0 < s1) load_tile(s0, vn);
    for (int sl = s0; sl < s1; ++sl) {
        if constexpr (PF) {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = vn[e];
            if (sl + 1 < s1) load_tile(sl + 1, vn);
        } else {
            load_tile(sl, v);
        }
        const cpx<T> *es = ell + (int64_t)(slot0 + sl) * nc;
        if constexpr (EARLY) {
            cpx<T> el[EH];
#pragma unroll
            for (int h = 0; h < EH; ++h) {
                const int64_t a = kept_pos(h);
                el[h] = a < n ? es[a] : cpx<T>{0, 0};
            }
            const cpx<T> elm = amid < n ? es[amid] : cpx<T>{0, 0};
            F::inverse(v, lds, twL2);
#pragma unroll
            for (int h = 0; h < EH; ++h) acc[h] = cadd(acc[h], cdiag(el[h], v[(h / RH) * RF + h % RH]));
            accm = cadd(accm, cdiag(elm, v[RH]));
        } else {
            F::inverse(v, lds, twL2);
#pragma unroll
            for (int h = 0; h < EH; ++h) {
                const int64_t a = kept_pos(h);
                if (a < n) acc[h] = cadd(acc[h], cdiag(es[a], v[(h / RH) * RF + h % RH]));
            }
            if (amid < n) accm = cadd(accm, cdiag(es[amid], v[RH]));
        }
    }
    cpx<T> *Wg = W + ((int64_t)(gofs + g) * batch + b) * nc;
#pragma unroll
    for (int h = 0; h < EH; ++h) {
        const int64_t a = kept_pos(h);
        if (a < n) Wg[a] = acc[h];
    }
    if (amid < n) Wg[amid] = accm;
}

// Column lengths built for a row length: L1 L2 <= MP_LMAX, and for the
// double-precision rows of 8192 points only columns of 256 and 512
template <typename T, int L1, int L2>
constexpr bool mp_cols_built()
{
    return (int64_t)L1 * L2 <= MP_LMAX && (L1 != mp_row_xl<T>() || L2 == 256 || L2 == 512);
}

// Column lengths instantiated for each row length (L1 L2 <= MP_LMAX).
#define THX_L2_CASES(X) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) \
    X(10) X(20) X(40) X(80) X(160) X(320) X(640) \
    X(6) X(12) X(24) X(48) X(96) X(192) X(384) X(768)

template <typename T, int L1>
bool mp_p1_l2(const MultiPassGeom &g, const void *X, int64_t nc, int64_t n, const void *ell, int slot0,
              int nslots, int spb, const void *src, void *U, int64_t batch, const void *twL2, const void *twA,
              hipStream_t s, const AlphaIn &ain)
{
    const int nsg = (nslots + spb - 1) / spb;
    switch (g.L2) {
#define THX_P1(LL2)                                                                                       \
    case LL2:                                                                                             \
        if constexpr (mp_cols_built<T, L1, LL2>()) {                                                     \
            const dim3 grid((unsigned)(L1 / mp_tc<T, LL2>() * nsg * batch));                               \
            if (spb > 1)                                                                                  \
                k_mp_p1<T, L1, LL2, true><<<grid, mp_nt<T, LL2>(), 0, s>>>(                               \
                    (const cpx<T> *)X, nc, n, (const cpx<T> *)ell, slot0, nslots, spb,                    \
                    (const cpx<T> *)src, (cpx<T> *)U, batch, (const cpx<T> *)twL2, (const cpx<T> *)twA,   \
                    ain);                                                                                 \
            else                                                                                          \
                k_mp_p1<T, L1, LL2, false><<<grid, mp_nt<T, LL2>(), 0, s>>>(                              \
                    (const cpx<T> *)X, nc, n, (const cpx<T> *)ell, slot0, nslots, 1,                      \
                    (const cpx<T> *)src, (cpx<T> *)U, batch, (const cpx<T> *)twL2, (const cpx<T> *)twA,   \
                    ain);                                                                                 \
            return true;                                                                                  \
        } else {                                                                                          \
            return false;                                                                                 \
        }
        THX_L2_CASES(THX_P1)
#undef THX_P1
    default: return false;
    }
}

template <typename T>
bool launch_mp_p1(const MultiPassGeom &g, const void *X, int64_t nc, int64_t n, const void *ell,
                  int slot0, int nslots, int spb, const void *src, void *U, int64_t batch, const void *twL2,
                  const void *twA, hipStream_t s, const AlphaIn *ainp)
{
    if (ell && (n > g.L1 * g.L2 / 2 + 1 || n > nc)) return false; // zero padding above L/2 is assumed
    if (spb < 1 || nslots < 1 || (spb > 1 && !ell)) return false;
    if (ell && !X && !(ainp && ainp->alpha)) return false; // input lanes: packed X or the vector
    AlphaIn ain{};
    if (ainp && ell) ain = *ainp;
    if (g.L1 == mp_row_short<T>())
        return mp_p1_l2<T, (int)mp_row_short<T>()>(g, X, nc, n, ell, slot0, nslots, spb, src, U, batch, twL2,
                                                    twA, s, ain);
    if (g.L1 == mp_row_long<T>())
        return mp_p1_l2<T, (int)mp_row_long<T>()>(g, X, nc, n, ell, slot0, nslots, spb, src, U, batch, twL2,
                                                   twA, s, ain);
    if constexpr (mp_row_xl<T>() > 0)
        if (g.L1 == mp_row_xl<T>())
            return mp_p1_l2<T, (int)mp_row_xl<T>()>(g, X, nc, n, ell, slot0, nslots, spb, src, U, batch, twL2,
                                                     twA, s, ain);
    return false;
}
template bool launch_mp_p1<double>(const MultiPassGeom &, const void *, int64_t, int64_t, const void *, int, int, int, const void *, void *, int64_t, const void *, const void *, hipStream_t, const AlphaIn *);
template bool launch_mp_p1<float>(const MultiPassGeom &, const void *, int64_t, int64_t, const void *, int, int, int, const void *, void *, int64_t, const void *, const void *, hipStream_t, const AlphaIn *);

template <typename T, int L1>
void mp_p2_run(const MultiPassGeom &g, void *U, int nslots, int64_t batch, const void *that_perm,
               const void *twL1, const void *twA, const void *twL2, bool full, void *out, double scale,
               hipStream_t s)
{
    dim3 grid((unsigned)(g.L2 * nslots * batch));
    k_mp_p2<T, L1><<<grid, p2_threads<T, L1>(), 0, s>>>(
        (cpx<T> *)U, (int)g.L2, (int)(nslots * batch), (const cpx<T> *)that_perm, (const cpx<T> *)twL1,
        (const cpx<T> *)twA, (const cpx<T> *)twL2, full ? 1 : 0, (cpx<T> *)out, (T)scale);
}

template <typename T>
bool launch_mp_p2(const MultiPassGeom &g, void *U, int nslots, int64_t batch, const void *that_perm,
                  const void *twL1, const void *twA, const void *twL2, bool full, void *out,
                  double scale, hipStream_t s)
{
    if (g.L2 < 2 || g.L2 > 1024 || g.L1 * g.L2 > MP_LMAX) return false;
    if (g.L1 == mp_row_short<T>())
        mp_p2_run<T, (int)mp_row_short<T>()>(g, U, nslots, batch, that_perm, twL1, twA, twL2, full, out, scale, s);
    else if (g.L1 == mp_row_long<T>())
        mp_p2_run<T, (int)mp_row_long<T>()>(g, U, nslots, batch, that_perm, twL1, twA, twL2, full, out, scale, s);
    else if constexpr (mp_row_xl<T>() > 0) {
        if (g.L1 != mp_row_xl<T>() || (g.L2 != 256 && g.L2 != 512)) return false;
        mp_p2_run<T, (int)mp_row_xl<T>()>(g, U, nslots, batch, that_perm, twL1, twA, twL2, full, out, scale, s);
    } else
        return false;
    return true;
}
template bool launch_mp_p2<double>(const MultiPassGeom &, void *, int, int64_t, const void *, const void *, const void *, const void *, bool, void *, double, hipStream_t);
template bool launch_mp_p2<float>(const MultiPassGeom &, void *, int, int64_t, const void *, const void *, const void *, const void *, bool, void *, double, hipStream_t);

template <typename T, int L1>
bool mp_p2f_l2(const MultiPassGeom &g, const void *X, int64_t nc, int64_t n, const void *ell, int slot0,
               int nslots, void *U, int64_t batch, const void *that_perm, const void *twL1, const void *twA,
               const void *twL2, hipStream_t s)
{
    const int64_t items = ((int64_t)nslots * batch + 7) / 8 * 8;
    switch (g.L2) {
#define THX_P2F(LL2)                                                                                     \
    case LL2:                                                                                            \
        k_mp_p2f<T, L1, LL2><<<dim3((unsigned)(items * LL2)), p2_threads<T, L1>(), 0, s>>>(             \
            (const cpx<T> *)X, nc, n, (const cpx<T> *)ell, slot0, nslots, (cpx<T> *)U, batch,            \
            (const cpx<T> *)that_perm, (const cpx<T> *)twL1, (const cpx<T> *)twA, (const cpx<T> *)twL2); \
        return true;
        THX_P2F(2) THX_P2F(4)
#undef THX_P2F
    default: return false;
    }
}

template <typename T>
bool launch_mp_p2f(const MultiPassGeom &g, const void *X, int64_t nc, int64_t n, const void *ell, int slot0,
                   int nslots, void *U, int64_t batch, const void *that_perm, const void *twL1, const void *twA,
                   const void *twL2, hipStream_t s)
{
    if (n > g.L1 * g.L2 / 2 + 1 || n > nc || nslots < 1) return false; // zero padding above L/2 is assumed
    if ((int64_t)nslots * batch * g.L2 + 8 * g.L2 > ((int64_t)1 << 31) - 1) return false;
    if (g.L1 == mp_row_short<T>())
        return mp_p2f_l2<T, (int)mp_row_short<T>()>(g, X, nc, n, ell, slot0, nslots, U, batch, that_perm, twL1,
                                                     twA, twL2, s);
    if (g.L1 == mp_row_long<T>())
        return mp_p2f_l2<T, (int)mp_row_long<T>()>(g, X, nc, n, ell, slot0, nslots, U, batch, that_perm, twL1,
                                                    twA, twL2, s);
    return false;
}
template bool launch_mp_p2f<double>(const MultiPassGeom &, const void *, int64_t, int64_t, const void *, int, int, void *, int64_t, const void *, const void *, const void *, const void *, hipStream_t);
template bool launch_mp_p2f<float>(const MultiPassGeom &, const void *, int64_t, int64_t, const void *, int, int, void *, int64_t, const void *, const void *, const void *, const void *, hipStream_t);

template <typename T, int L1>
bool mp_p3_l2(const MultiPassGeom &g, const void *U, int64_t nc, int64_t n, const void *ell, int slot0,
              int nslots, int spg, int G, void *Wpart, int gofs, int64_t batch, const void *twL2,
              hipStream_t s)
{
    switch (g.L2) {
#define THX_P3(LL2)                                                                                   \
    case LL2:                                                                                         \
        if constexpr (mp_cols_built<T, L1, LL2>()) {                                                 \
            k_mp_p3<T, L1, LL2><<<dim3((unsigned)(L1 / mp_tc<T, LL2>()), (unsigned)G, (unsigned)batch), \
                                  mp_nt<T, LL2>(), 0, s>>>((const cpx<T> *)U, nc, n,                  \
                                                           (const cpx<T> *)ell, slot0, nslots, spg,   \
                                                           (cpx<T> *)Wpart, gofs, batch,              \
                                                           (const cpx<T> *)twL2);                     \
            return true;                                                                              \
        } else {                                                                                      \
            return false;                                                                             \
        }
        THX_L2_CASES(THX_P3)
#undef THX_P3
    default: return false;
    }
}

template <typename T>
bool launch_mp_p3(const MultiPassGeom &g, const void *U, int64_t nc, int64_t n, const void *ell,
                  int slot0, int nslots, int spg, int G, void *Wpart, int gofs, int64_t batch,
                  const void *twL2, hipStream_t s)
{
    if (n > g.L1 * g.L2 / 2 + 1 || n > nc) return false; // the kernel keeps outputs below L/2 + 1 only
    if (g.L1 == mp_row_short<T>())
        return mp_p3_l2<T, (int)mp_row_short<T>()>(g, U, nc, n, ell, slot0, nslots, spg, G, Wpart, gofs, batch, twL2, s);
    if (g.L1 == mp_row_long<T>())
        return mp_p3_l2<T, (int)mp_row_long<T>()>(g, U, nc, n, ell, slot0, nslots, spg, G, Wpart, gofs, batch, twL2, s);
    if constexpr (mp_row_xl<T>() > 0)
        if (g.L1 == mp_row_xl<T>())
            return mp_p3_l2<T, (int)mp_row_xl<T>()>(g, U, nc, n, ell, slot0, nslots, spg, G, Wpart, gofs, batch,
                                                     twL2, s);
    return false;
}
template bool launch_mp_p3<double>(const MultiPassGeom &, const void *, int64_t, int64_t, const void *, int, int, int, int, void *, int, int64_t, const void *, hipStream_t);
template bool launch_mp_p3<float>(const MultiPassGeom &, const void *, int64_t, int64_t, const void *, int, int, int, int, void *, int, int64_t, const void *, hipStream_t);

} // namespace thx
