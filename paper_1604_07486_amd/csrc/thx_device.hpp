// thx_device.hpp -- complex arithmetic on interleaved (re, im) pairs for the
// libthx kernels (gfx950 / CDNA4).
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

// A workgroup-uniform pointer the compiler must treat as changed: loads through
// it are not hoisted out of the enclosing loop (keeps register pressure down
// where re-reading from cache is cheaper than holding the values).
template <typename P>
__device__ __forceinline__ P *opaque_ptr(P *p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// Streaming (nontemporal) access to data touched once per pass, so that L2
// keeps the reused tiles (symbol rows, packed input).
#ifndef THX_NT
#define THX_NT 1
#endif
template <typename T>
__device__ __forceinline__ cpx<T> ld_stream(const cpx<T> *p)
{
    if constexpr (THX_NT) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
        return cpx<T>{v.x, v.y};
    } else {
        return *p;
    }
}
template <typename T>
__device__ __forceinline__ void st_stream(cpx<T> *p, cpx<T> a)
{
    if constexpr (THX_NT) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        v2 v;
        v.x = a.x;
        v.y = a.y;
        __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
    } else {
        *p = a;
    }
}

} // namespace thx
