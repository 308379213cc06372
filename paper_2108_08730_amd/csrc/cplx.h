// Small complex helpers for the device code (interleaved re/im pairs).
#pragma once
#include <hip/hip_runtime.h>

namespace h27 {

template <typename R> struct V2;
template <> struct V2<float>  { using T = float2; };
template <> struct V2<double> { using T = double2; };

template <typename R>
struct Cx {
    R re, im;
};

template <typename R> __device__ __forceinline__ Cx<R> mk(R re, R im) { return Cx<R>{re, im}; }
template <typename R> __device__ __forceinline__ Cx<R> zero() { return Cx<R>{R(0), R(0)}; }
template <typename R> __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
// acc += a * b (complex)
template <typename R> __device__ __forceinline__ void cmac(Cx<R>& acc, Cx<R> a, Cx<R> b) {
    acc.re += a.re * b.re - a.im * b.im;
    acc.im += a.re * b.im + a.im * b.re;
}
// acc += s * b (real s)
template <typename R> __device__ __forceinline__ void rmac(Cx<R>& acc, R s, Cx<R> b) {
    acc.re += s * b.re;
    acc.im += s * b.im;
}
template <typename R> __device__ __forceinline__ Cx<R> cinv(Cx<R> a) {
    R d = R(1) / (a.re * a.re + a.im * a.im);
    return {a.re * d, -a.im * d};
}
template <typename R> __device__ __forceinline__ Cx<R> ld(const typename V2<R>::T* p) {
    typename V2<R>::T v = *p;
    return {v.x, v.y};
}
template <typename R> __device__ __forceinline__ void st(typename V2<R>::T* p, Cx<R> a) {
    typename V2<R>::T v;
    v.x = a.re;
    v.y = a.im;
    *p = v;
}
// streaming (non-temporal) access for data touched once: it does not evict
// reused data from the caches
template <typename R> using NtV2 = R __attribute__((ext_vector_type(2)));
template <typename R> __device__ __forceinline__ Cx<R> ld_nt(const typename V2<R>::T* p) {
    const NtV2<R> v = __builtin_nontemporal_load(reinterpret_cast<const NtV2<R>*>(p));
    return {v.x, v.y};
}
template <typename R> __device__ __forceinline__ void st_nt(typename V2<R>::T* p, Cx<R> a) {
    NtV2<R> v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, reinterpret_cast<NtV2<R>*>(p));
}
// XCD-contiguous block order for a grid of one point per thread: block b runs
// on XCD b % 8 (blocks are dispatched round robin over the eight XCDs), so
// logical block xcd * (nb / 8) + ... gives each XCD a contiguous range of
// points and the neighbouring rows and planes a block reads are ones its own
// XCD's L2 has just fetched
__device__ __forceinline__ int64_t xcd_block() {
    const int nb = static_cast<int>(gridDim.x), bx = static_cast<int>(blockIdx.x);
    const int xcd = bx & 7, q8 = nb >> 3, r8 = nb & 7;
    return static_cast<int64_t>(xcd) * q8 + (xcd < r8 ? xcd : r8) + (bx >> 3);
}

}  // namespace h27
