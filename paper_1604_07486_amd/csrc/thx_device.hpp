// thx_device.hpp -- device building blocks for libthx (gfx950 / CDNA4).
//
// Complex arithmetic on interleaved (re, im) pairs and a workgroup-level
// Stockham FFT held in LDS.  The FFT runs `NB` interleaved sequences of
// length M at once (element i of sequence c at buf[i*NB + c]), which is the
// layout of a column tile of a row-major matrix: it serves both the single
// row transforms (NB = 1) and the column passes of the four-step FFT.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace thx {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// componentwise product: the two real sub-problems packed in (re, im) are
// scaled by their own diagonals
template <typename T>
__device__ __forceinline__ cpx<T> cdiag(cpx<T> d, cpx<T> v) { return {d.x * v.x, d.y * v.y}; }

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Radix-R butterflies (R = 2, 4) of the DFT with kernel exp(-+2 pi i / R).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T> *v)
{
    if constexpr (R == 2) {
        cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else {
        cpx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        cpx<T> a2 = cadd(v[1], v[3]), a3 = csub(v[1], v[3]);
        // forward: y1 = a1 - i a3, y3 = a1 + i a3; inverse swaps them
        cpx<T> mi = {a3.y, -a3.x}; // -i * a3
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        if constexpr (!INV) {
            v[1] = cadd(a1, mi);
            v[3] = csub(a1, mi);
        } else {
            v[1] = csub(a1, mi);
            v[3] = cadd(a1, mi);
        }
    }
}

// One Stockham (autosort) stage of radix R after sub-transforms of size Ns:
// butterfly j reads x[j + r M/R], twiddles by w_{Ns R}^{(j mod Ns) r}, and
// writes y[(j/Ns) Ns R + (j mod Ns) + r Ns].  All reads of the stage complete
// (barrier) before any write, so the stage runs in place.
// tw[k] = exp(-2 pi i k / M), k < M.
template <typename T, int M, int NB, int NT, bool INV, int R, int Ns>
__device__ __forceinline__ void fft_stage(cpx<T> *buf, const cpx<T> *__restrict__ tw)
{
    constexpr int NBF = (M / R) * NB;
    constexpr int PER = (NBF + NT - 1) / NT;
    cpx<T> v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int w = (int)threadIdx.x + p * NT;
        if (NBF % NT == 0 || w < NBF) {
            const int c = w % NB, j = w / NB, k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[p][r] = buf[(j + r * (M / R)) * NB + c];
            if constexpr (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const cpx<T> t = tw[k * r * (M / (Ns * R))];
                    v[p][r] = INV ? cmulc(v[p][r], t) : cmul(v[p][r], t);
                }
            }
            dft<T, R, INV>(v[p]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int w = (int)threadIdx.x + p * NT;
        if (NBF % NT == 0 || w < NBF) {
            const int c = w % NB, j = w / NB, k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[(base + r * Ns) * NB + c] = v[p][r];
        }
    }
    __syncthreads();
}

template <typename T, int M, int NB, int NT, bool INV, int Ns>
__device__ __forceinline__ void fft_stages(cpx<T> *buf, const cpx<T> *__restrict__ tw)
{
    if constexpr (Ns < M) {
        // one radix-2 stage when the remaining length is an odd power of two
        constexpr int R = (ilog2(M / Ns) % 2 == 1) ? 2 : 4;
        fft_stage<T, M, NB, NT, INV, R, Ns>(buf, tw);
        fft_stages<T, M, NB, NT, INV, Ns * R>(buf, tw);
    }
}

// Unnormalised DFT of length M (forward kernel exp(-2 pi i/M), inverse
// exp(+2 pi i/M)) of NB interleaved sequences in LDS.  Entry and exit are
// barrier-synchronised: the caller may read any element afterwards.
template <typename T, int M, int NB, int NT, bool INV>
__device__ __forceinline__ void lds_fft(cpx<T> *buf, const cpx<T> *__restrict__ tw)
{
    static_assert((M & (M - 1)) == 0 && M >= 2, "power-of-two length");
    fft_stages<T, M, NB, NT, INV, 1>(buf, tw);
}

} // namespace thx
