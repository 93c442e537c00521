// fft_reg.hpp -- register-resident Stockham FFT for one workgroup (gfx950).
//
// A workgroup of NT threads transforms NB interleaved sequences of length M
// (sequence c, element i at logical position i*NB + c).  Each thread keeps
// E = M*NB/NT complex values in registers.  The transform is a sequence of
// radix-R stages (R = RMAX while possible, then one stage of 2, 4 or 8, and a
// radix-3 or radix-5 stage for M = 3 * 2^m or 5 * 2^m); the inverse runs the
// radices in reverse order.  Between stages the values are
// exchanged through LDS (padded one slot per 16 to spread the banks); the
// first stage reads its inputs from registers and the last stage leaves its
// outputs in registers, so callers load and store global memory directly in
// the stage layouts, which are coalesced:
//
//   input layout of a forward transform (= output layout of an inverse):
//       v[p*R1 + r] holds position j + r*(M/R1) of sequence c
//   output layout of a forward transform (= input layout of an inverse):
//       v[p*RS + q] holds position j + q*(M/RS) of sequence c
//   where w = threadIdx.x + NT*p, c = w % NB, j = w / NB, R1 / RS are the
//   first / last forward radices.
//
// Stage with radix R after sub-transforms of size Ns: butterfly j reads
// x[j + r M/R], multiplies by w_{Ns R}^{(j mod Ns) r}, applies the radix-R DFT
// and writes y[(j/Ns) Ns R + (j mod Ns) + q Ns]  (Stockham autosort).
#pragma once
#include "thx_device.hpp"

namespace thx {

// Lengths are M = 2^m, 3 * 2^m or 5 * 2^m.  Forward radices of stage s for
// largest power-of-two radix RMAX (16, 8 or 4): RMAX, RMAX, ..., the
// power-of-two remainder, then one radix-3 or radix-5 stage when 3 or 5 divides
// M (last forward, first inverse, so the first forward radix stays a power of
// two whenever M has a power-of-two factor).
constexpr int odd_part(int M) { return M % 3 == 0 ? 3 : (M % 5 == 0 ? 5 : 1); }
constexpr int pow2_part(int M) { return M / odd_part(M); }
constexpr int nstages2(int P, int RMAX) { return ilog2(P) / ilog2(RMAX) + (ilog2(P) % ilog2(RMAX) ? 1 : 0); }
constexpr int nstages(int M, int RMAX) { return nstages2(pow2_part(M), RMAX) + (odd_part(M) > 1 ? 1 : 0); }
constexpr int fwd_radix(int M, int s, int RMAX)
{
    const int P = pow2_part(M);
    return s >= nstages2(P, RMAX) ? odd_part(M)
                                  : ((s < ilog2(P) / ilog2(RMAX)) ? RMAX : (1 << (ilog2(P) % ilog2(RMAX))));
}
template <bool INV>
constexpr int stage_radix(int M, int s, int RMAX)
{
    return INV ? fwd_radix(M, nstages(M, RMAX) - 1 - s, RMAX) : fwd_radix(M, s, RMAX);
}
// product of the radices before stage s
template <bool INV>
constexpr int stage_ns(int M, int s, int RMAX)
{
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= stage_radix<INV>(M, i, RMAX);
    return ns;
}
// threads for M*NB points with at least min(M, RMAX) values per thread
// (power-of-two M)
constexpr int fft_threads(int M, int NB, int RMAX, int maxnt = 1024)
{
    return (M * NB / (M < RMAX ? M : RMAX)) > maxnt ? maxnt : (M * NB / (M < RMAX ? M : RMAX));
}

#ifndef THX_LDS_PAD
#define THX_LDS_PAD 1
#endif
__device__ __forceinline__ int lds_pad(int i) { return THX_LDS_PAD ? i + (i >> 4) : i; }
constexpr int lds_padded(int n) { return THX_LDS_PAD ? n + (n >> 4) : n; }
// For b >= 0 and a stride S that is a multiple of 16, the padded index of
// b + k S is lds_pad(b) + k lds_padded(S): the elements a thread moves in one
// exchange then sit at constant offsets from one base address, and the
// compiler folds them into the LDS instructions' offset fields.
constexpr bool lds_linear(int S) { return !THX_LDS_PAD || S % 16 == 0; }

// w_R^m = exp(-+ 2 pi i m / R) for the constant twiddles inside a radix-R DFT
template <typename T, int R, int m, bool INV>
__device__ __forceinline__ cpx<T> wconst()
{
    constexpr int mm = ((m % R) + R) % R;
    // cos / sin of 2 pi mm / R for R | 16
    constexpr int e = mm * (16 / R); // in units of 2 pi / 16
    constexpr double C[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                              0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
    constexpr double S[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                              1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};
    return cpx<T>{(T)C[e], (T)(INV ? S[e] : -S[e])};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cpx<T> &a, cpx<T> &b)
{
    const cpx<T> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// in-place radix-4 DFT of (a, b, c, d) = x[0..3]
template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T> &x0, cpx<T> &x1, cpx<T> &x2, cpx<T> &x3)
{
    const cpx<T> a0 = cadd(x0, x2), a1 = csub(x0, x2);
    const cpx<T> a2 = cadd(x1, x3), a3 = csub(x1, x3);
    const cpx<T> mi = {a3.y, -a3.x}; // -i a3
    x0 = cadd(a0, a2);
    x2 = csub(a0, a2);
    if constexpr (!INV) {
        x1 = cadd(a1, mi);
        x3 = csub(a1, mi);
    } else {
        x1 = csub(a1, mi);
        x3 = cadd(a1, mi);
    }
}

// radix-3 DFT: with s = x1 + x2, d = x1 - x2, y0 = x0 + s and
// y1,2 = x0 - s/2 -+ i (sqrt(3)/2) d (forward; signs swapped for the inverse)
template <typename T, bool INV>
__device__ __forceinline__ void dft3(cpx<T> &x0, cpx<T> &x1, cpx<T> &x2)
{
    constexpr T h = (T)0.86602540378443864676; // sqrt(3)/2
    const cpx<T> sm = cadd(x1, x2), df = csub(x1, x2);
    const cpx<T> t = {x0.x - (T)0.5 * sm.x, x0.y - (T)0.5 * sm.y};
    const cpx<T> r = INV ? cpx<T>{-h * df.y, h * df.x} : cpx<T>{h * df.y, -h * df.x}; // -+ i h d
    x0 = cadd(x0, sm);
    x1 = cadd(t, r);
    x2 = csub(t, r);
}

// radix-5 DFT: with c_m = cos(2 pi m / 5), s_m = sin(2 pi m / 5),
// t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4, t4 = x2 - x3,
//   y0 = x0 + t1 + t2,
//   y1,4 = (x0 + c1 t1 + c2 t2) -+ i (s1 t3 + s2 t4),
//   y2,3 = (x0 + c2 t1 + c1 t2) -+ i (s2 t3 - s1 t4)
// (forward; the signs of the imaginary terms swap for the inverse)
template <typename T, bool INV>
__device__ __forceinline__ void dft5(cpx<T> &x0, cpx<T> &x1, cpx<T> &x2, cpx<T> &x3, cpx<T> &x4)
{
    constexpr T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    constexpr T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    const cpx<T> t1 = cadd(x1, x4), t2 = cadd(x2, x3), t3 = csub(x1, x4), t4 = csub(x2, x3);
    const cpx<T> a1 = {x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y};
    const cpx<T> a2 = {x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y};
    const cpx<T> b1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    const cpx<T> b2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    // -i b = (b.y, -b.x)
    const cpx<T> mb1 = INV ? cpx<T>{-b1.y, b1.x} : cpx<T>{b1.y, -b1.x};
    const cpx<T> mb2 = INV ? cpx<T>{-b2.y, b2.x} : cpx<T>{b2.y, -b2.x};
    x0 = {x0.x + t1.x + t2.x, x0.y + t1.y + t2.y};
    x1 = cadd(a1, mb1);
    x4 = csub(a1, mb1);
    x2 = cadd(a2, mb2);
    x3 = csub(a2, mb2);
}

// Radix-R DFT in registers, R = R1 * R2 with input n = R2 n1 + n2 and output
// k = k1 + R1 k2: DFT_R1 over n1, twiddle w_R^{n2 k1}, DFT_R2 over n2.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T> *v)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 3) {
        dft3<T, INV>(v[0], v[1], v[2]);
    } else if constexpr (R == 5) {
        dft5<T, INV>(v[0], v[1], v[2], v[3], v[4]);
    } else if constexpr (R == 2) {
        dft2<T, INV>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<T, INV>(v[0], v[1], v[2], v[3]);
    } else {
        constexpr int R1 = 4, R2 = R / 4; // R = 8: (4, 2); R = 16: (4, 4)
        cpx<T> y[R];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            cpx<T> a = v[n2], b = v[R2 + n2], c = v[2 * R2 + n2], d = v[3 * R2 + n2];
            dft4<T, INV>(a, b, c, d);
            y[0 * R2 + n2] = a;
            y[1 * R2 + n2] = b;
            y[2 * R2 + n2] = c;
            y[3 * R2 + n2] = d;
        }
        // twiddle y[k1][n2] *= w_R^{n2 k1}
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) {
#pragma unroll
            for (int n2 = 1; n2 < R2; ++n2) {
                cpx<T> w;
                // compile-time constant selection
                switch (n2 * k1) {
                case 1: w = wconst<T, R, 1, INV>(); break;
                case 2: w = wconst<T, R, 2, INV>(); break;
                case 3: w = wconst<T, R, 3, INV>(); break;
                case 4: w = wconst<T, R, 4, INV>(); break;
                case 6: w = wconst<T, R, 6, INV>(); break;
                case 9: w = wconst<T, R, 9, INV>(); break;
                default: w = cpx<T>{1, 0}; break;
                }
                y[k1 * R2 + n2] = cmul(y[k1 * R2 + n2], w);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            if constexpr (R2 == 2) {
                dft2<T, INV>(y[k1 * R2], y[k1 * R2 + 1]);
                v[k1] = y[k1 * R2];
                v[k1 + R1] = y[k1 * R2 + 1];
            } else {
                dft4<T, INV>(y[k1 * R2], y[k1 * R2 + 1], y[k1 * R2 + 2], y[k1 * R2 + 3]);
                v[k1] = y[k1 * R2];
                v[k1 + R1] = y[k1 * R2 + 1];
                v[k1 + 2 * R1] = y[k1 * R2 + 2];
                v[k1 + 3 * R1] = y[k1 * R2 + 3];
            }
        }
    }
}

// x times w (forward) or conj(w) (inverse)
template <typename T, bool INV>
__device__ __forceinline__ void twmul(cpx<T> &x, cpx<T> w)
{
    x = INV ? cmulc(x, w) : cmul(x, w);
}

// Twiddle factors w^r, r = 1..R-1, of one radix-R butterfly (w = w_M^{e1},
// from the table tw[e] = w_M^e, e < M): w^1, w^2, w^4, w^8 (as far as R needs
// them) come from pw(k) = w^(2^k) and every other power is a product of at most
// four of them; the factors are formed just before use to keep few registers
// live.
template <typename T, int R, bool INV, typename PW>
__device__ __forceinline__ void twiddle_products(cpx<T> *v, PW pw)
{
    const cpx<T> w1 = pw(0);
    twmul<T, INV>(v[1], w1);
    if constexpr (R == 2) return;
    const cpx<T> w2 = pw(1);
    twmul<T, INV>(v[2], w2);
    if constexpr (R == 3) return;
    const cpx<T> w3 = cmul(w1, w2);
    twmul<T, INV>(v[3], w3);
    if constexpr (R == 4) return;
    const cpx<T> w4 = pw(2);
    twmul<T, INV>(v[4], w4);
    if constexpr (R == 5) return;
    twmul<T, INV>(v[5], cmul(w1, w4));
    twmul<T, INV>(v[6], cmul(w2, w4));
    const cpx<T> w7 = cmul(w3, w4);
    twmul<T, INV>(v[7], w7);
    if constexpr (R == 8) return;
    const cpx<T> w8 = pw(3);
    twmul<T, INV>(v[8], w8);
    twmul<T, INV>(v[9], cmul(w1, w8));
    twmul<T, INV>(v[10], cmul(w2, w8));
    twmul<T, INV>(v[11], cmul(w3, w8));
    twmul<T, INV>(v[12], cmul(w4, w8));
    twmul<T, INV>(v[13], cmul(cmul(w1, w4), w8));
    twmul<T, INV>(v[14], cmul(cmul(w2, w4), w8));
    twmul<T, INV>(v[15], cmul(w7, w8));
}

// twiddles read from the table tw[e] = w_M^e where they are used
template <typename T, int R, bool INV>
__device__ __forceinline__ void apply_twiddles(cpx<T> *v, const cpx<T> *__restrict__ tw, int e1)
{
    // The exponent is made opaque so that the table reads stay here: hoisted out
    // of a caller's loop over ranks they would pin every stage's twiddles in
    // registers and force spills.
    asm volatile("" : "+v"(e1));
    twiddle_products<T, R, INV>(v, [&](int k) { return tw[e1 * (1 << k)]; });
}

// Table reads of one butterfly's twiddles issued ahead of their use
// (apply_loaded_twiddles then forms the products from them).
template <int R> constexpr int tw_reads() { return R == 2 ? 1 : (R <= 4 ? 2 : (R <= 8 ? 3 : 4)); }

template <typename T, int R>
__device__ __forceinline__ void load_twiddles(cpx<T> *w, const cpx<T> *__restrict__ tw, int e1)
{
    asm volatile("" : "+v"(e1));
#pragma unroll
    for (int k = 0; k < tw_reads<R>(); ++k) w[k] = tw[e1 * (1 << k)];
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void apply_loaded_twiddles(cpx<T> *v, const cpx<T> *w)
{
    twiddle_products<T, R, INV>(v, [&](int k) { return w[k]; });
}

// PREF: each stage issues the table reads of the next stage's twiddles before
// its own exchange and arithmetic, so that their latency is hidden behind them
// (costs the registers that hold them; off by default).
template <typename T, int M, int NB, int NT, int RMAX = 16, bool PREF = false>
struct RegFFT {
    static constexpr int E = M * NB / NT;
    static constexpr int NS = nstages(M, RMAX);
    static constexpr int R_FIRST = fwd_radix(M, 0, RMAX);
    static constexpr int R_LAST = fwd_radix(M, NS - 1, RMAX);
    static constexpr int LDS = lds_padded(M * NB);
    static_assert(E * NT == M * NB, "elements per thread");
    static_assert((pow2_part(M) & (pow2_part(M) - 1)) == 0, "length 2^m, 3 * 2^m or 5 * 2^m");

    // logical position (i*NB + c) of register slot `slot` in the forward input layout
    __device__ static __forceinline__ void in_pos(int slot, int &pos, int &c)
    {
        const int p = slot / R_FIRST, r = slot % R_FIRST;
        const int w = (int)threadIdx.x + NT * p;
        c = w % NB;
        pos = w / NB + r * (M / R_FIRST);
    }
    // logical position in the forward output layout
    __device__ static __forceinline__ void out_pos(int slot, int &pos, int &c)
    {
        const int p = slot / R_LAST, q = slot % R_LAST;
        const int w = (int)threadIdx.x + NT * p;
        c = w % NB;
        pos = w / NB + q * (M / R_LAST);
    }

    // table reads of one thread's twiddles in stage s (at least one slot)
    template <bool INV, int s>
    static constexpr int stage_tw_reads()
    {
        if constexpr (s >= NS) return 1;
        else return (E / stage_radix<INV>(M, s, RMAX)) * tw_reads<stage_radix<INV>(M, s, RMAX)>();
    }
    template <bool INV, int s>
    __device__ static __forceinline__ void load_stage_twiddles(cpx<T> *w, const cpx<T> *__restrict__ tw)
    {
        constexpr int R = stage_radix<INV>(M, s, RMAX);
        constexpr int Ns = stage_ns<INV>(M, s, RMAX);
#pragma unroll
        for (int p = 0; p < E / R; ++p) {
            const int j = ((int)threadIdx.x + NT * p) / NB;
            load_twiddles<T, R>(w + p * tw_reads<R>(), tw, (j % Ns) * (M / (Ns * R)));
        }
    }

    // `wpre`: this stage's twiddle reads, issued by the previous stage (PREF)
    template <bool INV, int s>
    __device__ static __forceinline__ void stages(cpx<T> *v, cpx<T> *lds, const cpx<T> *__restrict__ tw,
                                                  const cpx<T> *wpre)
    {
        if constexpr (s < NS) {
            constexpr int R = stage_radix<INV>(M, s, RMAX);
            constexpr int Ns = stage_ns<INV>(M, s, RMAX);
            constexpr int PB = E / R; // butterflies per thread
            static_assert(PB * R == E, "radix divides the per-thread count");
            cpx<T> wnext[stage_tw_reads<INV, s + 1>()];
            if constexpr (PREF && s + 1 < NS) load_stage_twiddles<INV, s + 1>(wnext, tw);
            if constexpr (s > 0) {
                // values are in LDS at the positions written by the previous stage
#pragma unroll
                for (int p = 0; p < PB; ++p) {
                    const int w = (int)threadIdx.x + NT * p;
                    const int c = w % NB, j = w / NB;
                    constexpr int S = (M / R) * NB; // position j + r M / R of sequence c
                    if constexpr (lds_linear(S)) {
                        const cpx<T> *src = lds + lds_pad(j * NB + c);
#pragma unroll
                        for (int r = 0; r < R; ++r) v[p * R + r] = src[r * lds_padded(S)];
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r) v[p * R + r] = lds[lds_pad(j * NB + c + r * S)];
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int p = 0; p < PB; ++p) {
                const int w = (int)threadIdx.x + NT * p;
                const int j = w / NB;
                if constexpr (Ns > 1) {
                    if constexpr (PREF) apply_loaded_twiddles<T, R, INV>(v + p * R, wpre + p * tw_reads<R>());
                    else apply_twiddles<T, R, INV>(v + p * R, tw, (j % Ns) * (M / (Ns * R)));
                }
                dft<T, R, INV>(v + p * R);
            }
            if constexpr (s + 1 < NS) {
#pragma unroll
                for (int p = 0; p < PB; ++p) {
                    const int w = (int)threadIdx.x + NT * p;
                    const int c = w % NB, j = w / NB;
                    const int base = (j / Ns) * Ns * R + (j % Ns);
                    constexpr int S = Ns * NB; // position base + q Ns of sequence c
                    if constexpr (lds_linear(S)) {
                        cpx<T> *dst = lds + lds_pad(base * NB + c);
#pragma unroll
                        for (int q = 0; q < R; ++q) dst[q * lds_padded(S)] = v[p * R + q];
                    } else {
#pragma unroll
                        for (int q = 0; q < R; ++q) lds[lds_pad(base * NB + c + q * S)] = v[p * R + q];
                    }
                }
                __syncthreads();
            }
            stages<INV, s + 1>(v, lds, tw, wnext);
        }
    }

    // forward: input layout -> output layout.  `lds` must hold LDS elements;
    // the caller needs no barrier before the call, and one before the next
    // use of `lds` only if it writes it itself.
    __device__ static __forceinline__ void forward(cpx<T> *v, cpx<T> *lds, const cpx<T> *__restrict__ tw)
    {
        stages<false, 0>(v, lds, tw, nullptr);
    }
    // inverse (unnormalised): output layout -> input layout
    __device__ static __forceinline__ void inverse(cpx<T> *v, cpx<T> *lds, const cpx<T> *__restrict__ tw)
    {
        stages<true, 0>(v, lds, tw, nullptr);
    }
};

} // namespace thx
