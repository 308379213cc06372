// Krylov, multigrid-transfer and precision-conversion kernels of the solver.
//
// Reductions (norms, multi-vector dot products) are two-stage and
// deterministic: every block writes one partial per (right-hand side, basis
// vector), reduced by a second kernel in a fixed order; no atomics.  Partial
// sums are carried in FP64 (the vectors themselves are FP32 or FP64).
// The GMRES Hessenberg / Givens / triangular-solve steps run on the device in
// FP64, one thread per right-hand side.
#include "krylov.h"

namespace h27 {

GraphRec*& graph_rec() {
    static thread_local GraphRec* rec = nullptr;
    return rec;
}

constexpr int kRedBlock = 256;

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block-wide sum of NV doubles per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* [NV][4] */) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k * 4 + w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = sh[k * 4 + 0] + sh[k * 4 + 1] + sh[k * 4 + 2] + sh[k * 4 + 3];
    }
    __syncthreads();
}

template <typename T>
__global__ void fill_zero_kernel(T* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = T{};
}

static unsigned grid_for(int64_t n, int per_thread = 4) {
    int64_t b = (n + static_cast<int64_t>(kRedBlock) * per_thread - 1) / (static_cast<int64_t>(kRedBlock) * per_thread);
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return static_cast<unsigned>(b);
}

int fill_zero(void* p, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return HELM27_OK;
    if (bytes % 16 == 0) {
        const int64_t n = bytes / 16;
        H27_CHECK_HIP(launch(fill_zero_kernel<double2>, dim3(grid_for(n)), dim3(kRedBlock), 0, s,
                             static_cast<double2*>(p), n));
    } else {
        const int64_t n = bytes / 4;
        H27_CHECK_HIP(launch(fill_zero_kernel<float>, dim3(grid_for(n)), dim3(kRedBlock), 0, s,
                             static_cast<float*>(p), n));
    }
    return HELM27_OK;
}

// y = d * v (complex) with a fixed operation order (explicit fused
// multiply-adds), so every kernel that forms the first Jacobi sweep
// omega D^-1 b from the stored omega D^-1 gets the same bits.
template <typename V>
__device__ __forceinline__ V dmul(V d, V v) {
    V y;
    y.x = fma(d.x, v.x, -(d.y * v.y));
    y.y = fma(d.x, v.y, d.y * v.x);
    return y;
}

template <typename R>
__global__ void fill_one_kernel(typename V2<R>::T* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        typename V2<R>::T o;
        o.x = R(1);
        o.y = R(0);
        p[i] = o;
    }
}

template <typename R>
int fill_one(void* p, int64_t n, hipStream_t s) {
    if (n <= 0) return HELM27_OK;
    H27_CHECK_HIP(launch(fill_one_kernel<R>, dim3(grid_for(n)), dim3(kRedBlock), 0, s,
                         static_cast<typename V2<R>::T*>(p), n));
    return HELM27_OK;
}
template int fill_one<float>(void*, int64_t, hipStream_t);
template int fill_one<double>(void*, int64_t, hipStream_t);

// y[rhs] = dinv * b[rhs] per point (the first damped-Jacobi sweep from a zero
// iterate, with dinv = omega D^-1 stored once per level)
template <typename R>
__global__ void dinv_scale_kernel(const typename V2<R>::T* __restrict__ dinv, const typename V2<R>::T* __restrict__ b,
                                  typename V2<R>::T* __restrict__ y, int64_t N) {
    const int rhs = blockIdx.y;
    const typename V2<R>::T* br = b + static_cast<int64_t>(rhs) * N;
    typename V2<R>::T* yr = y + static_cast<int64_t>(rhs) * N;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock)
        yr[i] = dmul(dinv[i], br[i]);
}

template <typename R>
int dinv_scale(const void* dinv, const void* b, void* y, int64_t N, int nrhs, hipStream_t s) {
    using V = typename V2<R>::T;
    H27_CHECK_HIP(launch(dinv_scale_kernel<R>, dim3(grid_for(N), nrhs), dim3(kRedBlock), 0, s,
                         static_cast<const V*>(dinv), static_cast<const V*>(b), static_cast<V*>(y), N));
    return HELM27_OK;
}
template int dinv_scale<float>(const void*, const void*, void*, int64_t, int, hipStream_t);
template int dinv_scale<double>(const void*, const void*, void*, int64_t, int, hipStream_t);

// b[s][lin_s] = amp_s / h^3 (paper Sec. 3.1: delta source on a grid node)
__global__ void inject_kernel(double2* __restrict__ b, int64_t N, const int64_t* __restrict__ lin,
                              const double2* __restrict__ amp, int nsrc, double inv_h3) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsrc) {
        double2 v;
        v.x = amp[s].x * inv_h3;
        v.y = amp[s].y * inv_h3;
        b[static_cast<int64_t>(s) * N + lin[s]] = v;
    }
}

int inject_sources(double2* b, int64_t N, const int64_t* d_lin, const double2* d_amp, int nsrc, double h,
                   hipStream_t s) {
    hipLaunchKernelGGL(inject_kernel, dim3((nsrc + 63) / 64), dim3(64), 0, s, b, N, d_lin, d_amp, nsrc,
                       1.0 / (h * h * h));
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

// ---------------------------------------------------------------------------
// partial[rhs][blk] = sum over the block's elements of |x|^2
template <typename R>
__global__ __launch_bounds__(kRedBlock) void norm2_partial_kernel(const typename V2<R>::T* __restrict__ x, int64_t N,
                                                                  double* __restrict__ partial) {
    __shared__ double sh[4];
    const int rhs = blockIdx.y;
    const typename V2<R>::T* xr = x + static_cast<int64_t>(rhs) * N;
    double acc[1] = {0.0};
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock) {
        const typename V2<R>::T v = xr[i];
        acc[0] += static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
    }
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(rhs) * gridDim.x + blockIdx.x] = acc[0];
}

// out[k] = sum_b partial[k][b], one block per k; optionally sqrt
__global__ void reduce_rows_kernel(const double* __restrict__ partial, int nb, double* __restrict__ out, int take_sqrt) {
    __shared__ double sh[4];
    double acc[1] = {0.0};
    const double* p = partial + static_cast<int64_t>(blockIdx.x) * nb;
    for (int b = threadIdx.x; b < nb; b += kRedBlock) acc[0] += p[b];
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = take_sqrt ? sqrt(acc[0]) : acc[0];
}

template <typename R>
int norms(const void* x, int64_t N, int nrhs, double* d_partial, int max_blocks, double* d_out, hipStream_t s) {
    unsigned nb = grid_for(N);
    if (nb > static_cast<unsigned>(max_blocks)) nb = max_blocks;
    hipLaunchKernelGGL(norm2_partial_kernel<R>, dim3(nb, nrhs), dim3(kRedBlock), 0, s,
                       static_cast<const typename V2<R>::T*>(x), N, d_partial);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(nrhs), dim3(kRedBlock), 0, s, d_partial, static_cast<int>(nb), d_out,
                       1);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int norms<float>(const void*, int64_t, int, double*, int, double*, hipStream_t);
template int norms<double>(const void*, int64_t, int, double*, int, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Selective second Gram-Schmidt pass: a right-hand side is orthogonalised a
// second time only if the first pass cancelled more than 1 - 1/sqrt(2) of its
// norm, ||w'|| < ||w|| / sqrt(2) (the "twice is enough" test of Kahan and
// Parlett, as used by Daniel, Gragg, Kaufman and Stewart, 1976).  The test
// runs on the device per right-hand side; without the gate every pass runs.
__device__ __forceinline__ bool second_pass(const double* nrm0, const double* nrm1, int rhs) {
    if (!nrm0) return true;
    return nrm1[rhs] * nrm1[rhs] * 2.0 < nrm0[rhs] * nrm0[rhs];
}

// Multi-vector dot products h[rhs][j] = sum_i conj(V_j[rhs][i]) w[rhs][i] for
// all j < J in one launch, plus |w|^2 in slot J when self_norm is set.  V is
// [m+1][nrhs][N]; partial is [nrhs][J + self_norm][nb] (complex as 2 doubles).
//
// One pass over the elements for up to 32 slots: the block's four wavefronts
// split the slots into G groups (slot j goes to group j mod G) and, when there
// are fewer than four slots, the element strips too (E = 4 / G parts).  A
// wavefront walks 64-element strips and, per pair of strips, issues the loads
// of all its slots and of w before it uses any of them (2 NK + 2 loads in
// flight); its FP64 accumulators stay in registers.  The four wavefronts read
// the same w strips, which the CU's cache serves after the first.  With the
// gate (nrm0, nrm1) a right-hand side that needs no second pass exits at once;
// the reduction kernel writes its zeros.
template <typename R, int NK>
__device__ __forceinline__ void mdot_wave(const typename V2<R>::T* const (&src)[8], const typename V2<R>::T* wr,
                                          int64_t N, int64_t s0, int64_t sstep, int lane, double (&acc)[16]) {
    using V = typename V2<R>::T;
    const int64_t nfull = N / 64;   // strips with 64 elements
    int64_t st = s0;
    for (; st + sstep < nfull; st += 2 * sstep) {
        const int64_t i0 = st * 64 + lane, i1 = (st + sstep) * 64 + lane;
        const V w0 = wr[i0], w1 = wr[i1];
        V a[NK], b[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            a[k] = src[k][i0];
            b[k] = src[k][i1];
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {   // conj(v) * w
            acc[2 * k] += static_cast<double>(a[k].x) * w0.x + static_cast<double>(a[k].y) * w0.y;
            acc[2 * k + 1] += static_cast<double>(a[k].x) * w0.y - static_cast<double>(a[k].y) * w0.x;
            acc[2 * k] += static_cast<double>(b[k].x) * w1.x + static_cast<double>(b[k].y) * w1.y;
            acc[2 * k + 1] += static_cast<double>(b[k].x) * w1.y - static_cast<double>(b[k].y) * w1.x;
        }
    }
    for (; st * 64 < N; st += sstep) {   // at most two strips, the last possibly partial
        const int64_t i0 = st * 64 + lane;
        if (i0 < N) {
            const V w0 = wr[i0];
            V a[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k) a[k] = src[k][i0];
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                acc[2 * k] += static_cast<double>(a[k].x) * w0.x + static_cast<double>(a[k].y) * w0.y;
                acc[2 * k + 1] += static_cast<double>(a[k].x) * w0.y - static_cast<double>(a[k].y) * w0.x;
            }
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kRedBlock) void mdot_partial_kernel(const typename V2<R>::T* __restrict__ V, int64_t vstride,
                                                                 int J, const typename V2<R>::T* __restrict__ w,
                                                                 int64_t N, double* __restrict__ partial, int self_norm,
                                                                 const double* __restrict__ nrm0,
                                                                 const double* __restrict__ nrm1) {
    using VT = typename V2<R>::T;
    __shared__ double sh[32 * 4 * 2];   // [slot][part][re, im]
    const int rhs = blockIdx.y;
    const int JS = J + self_norm;
    if (!second_pass(nrm0, nrm1, rhs)) return;
    const VT* wr = w + static_cast<int64_t>(rhs) * N;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int sb = 0; sb < JS; sb += 32) {
        const int ns = JS - sb < 32 ? JS - sb : 32;                  // slots of this pass
        const int G = ns >= 4 ? 4 : (ns >= 2 ? 2 : 1), E = 4 / G;    // slot groups, element parts
        const int g = wave % G, e = wave / G;
        const int nk = (ns - g + G - 1) / G;                         // slots of this wavefront
        const VT* src[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int j = sb + g + G * k;
            if (j >= sb + ns) j = sb + ns - 1;   // unused, kept in range
            src[k] = j < J ? V + static_cast<int64_t>(j) * vstride + static_cast<int64_t>(rhs) * N : wr;
        }
        double acc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        const int64_t s0 = static_cast<int64_t>(blockIdx.x) * E + e, sstep = static_cast<int64_t>(gridDim.x) * E;
        switch (nk) {
            case 1: mdot_wave<R, 1>(src, wr, N, s0, sstep, lane, acc); break;
            case 2: mdot_wave<R, 2>(src, wr, N, s0, sstep, lane, acc); break;
            case 3: mdot_wave<R, 3>(src, wr, N, s0, sstep, lane, acc); break;
            case 4: mdot_wave<R, 4>(src, wr, N, s0, sstep, lane, acc); break;
            case 5: mdot_wave<R, 5>(src, wr, N, s0, sstep, lane, acc); break;
            case 6: mdot_wave<R, 6>(src, wr, N, s0, sstep, lane, acc); break;
            case 7: mdot_wave<R, 7>(src, wr, N, s0, sstep, lane, acc); break;
            default: mdot_wave<R, 8>(src, wr, N, s0, sstep, lane, acc); break;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < nk) {
                const double re = wave_sum(acc[2 * k]), im = wave_sum(acc[2 * k + 1]);
                if (lane == 0) {
                    const int t = g + G * k;   // slot within the pass
                    sh[(t * 4 + e) * 2] = re;
                    sh[(t * 4 + e) * 2 + 1] = im;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < ns) {
            const int t = threadIdx.x;
            double re = 0.0, im = 0.0;
            for (int q = 0; q < E; ++q) {
                re += sh[(t * 4 + q) * 2];
                im += sh[(t * 4 + q) * 2 + 1];
            }
            double* p = partial + ((static_cast<int64_t>(rhs) * JS + sb + t) * gridDim.x + blockIdx.x) * 2;
            p[0] = re;
            p[1] = im;
        }
        __syncthreads();
    }
}

// h[rhs * ldh + j] = sum_b partial[rhs][j][b] for j < J (and hsum[...] += the
// same when hsum is given); slot J (self_norm) gives selfn[rhs] = sqrt of the
// real part.  One block per (rhs, slot), summed in a fixed order.
__global__ void mdot_reduce_kernel(const double* __restrict__ partial, int nb, int J, int self_norm,
                                   double2* __restrict__ h, double2* __restrict__ hsum, int ldh,
                                   double* __restrict__ selfn, const double* __restrict__ nrm0,
                                   const double* __restrict__ nrm1) {
    __shared__ double sh[8];
    const int JS = J + self_norm;
    const int rhs = blockIdx.x / JS, j = blockIdx.x % JS;
    double acc[2] = {0.0, 0.0};
    if (second_pass(nrm0, nrm1, rhs)) {   // a gated-off right-hand side sums to zero
        const double* p = partial + (static_cast<int64_t>(rhs) * JS + j) * nb * 2;
        for (int b = threadIdx.x; b < nb; b += kRedBlock) {
            acc[0] += p[2 * b];
            acc[1] += p[2 * b + 1];
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        if (j == J) {
            selfn[rhs] = sqrt(acc[0] > 0.0 ? acc[0] : 0.0);
            return;
        }
        double2* o = h + static_cast<int64_t>(rhs) * ldh + j;
        o->x = acc[0];
        o->y = acc[1];
        if (hsum) {
            double2* t = hsum + static_cast<int64_t>(rhs) * ldh + j;
            t->x += acc[0];
            t->y += acc[1];
        }
    }
}

template <typename R>
int mdot(const void* V, int64_t vstride, int J, const void* w, int64_t N, int nrhs, double* d_partial, int max_blocks,
         double2* d_h, double2* d_hsum, int ldh, hipStream_t s, double* d_selfnrm, const double* d_gate0,
         const double* d_gate1) {
    if (J <= 0 || J > ldh) return HELM27_EINVAL;
    unsigned nb = grid_for(N);
    if (nb > static_cast<unsigned>(max_blocks)) nb = max_blocks;
    const int self_norm = d_selfnrm ? 1 : 0;
    hipLaunchKernelGGL(mdot_partial_kernel<R>, dim3(nb, nrhs), dim3(kRedBlock), 0, s,
                       static_cast<const typename V2<R>::T*>(V), vstride, J,
                       static_cast<const typename V2<R>::T*>(w), N, d_partial, self_norm, d_gate0, d_gate1);
    hipLaunchKernelGGL(mdot_reduce_kernel, dim3(nrhs * (J + self_norm)), dim3(kRedBlock), 0, s, d_partial,
                       static_cast<int>(nb), J, self_norm, d_h, d_hsum, ldh, d_selfnrm, d_gate0, d_gate1);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int mdot<float>(const void*, int64_t, int, const void*, int64_t, int, double*, int, double2*, double2*, int,
                         hipStream_t, double*, const double*, const double*);
template int mdot<double>(const void*, int64_t, int, const void*, int64_t, int, double*, int, double2*, double2*, int,
                          hipStream_t, double*, const double*, const double*);

// w[rhs] -= sum_{j < J} V_j[rhs] * hc[rhs][j] where hc are the coefficients of
// the current pass (FP64 on the device, applied in the vector precision);
// with partial != null also partial[rhs][blk] = sum of |w_new|^2 over the
// block's elements (FP64).  With the gate (nrm0, nrm1) a right-hand side that
// needs no second pass keeps w and reports |w|^2 = nrm1^2 (block 0).
template <typename R>
__global__ __launch_bounds__(kRedBlock) void cgs_update_kernel(const typename V2<R>::T* __restrict__ V, int64_t vstride,
                                                               int J, const double2* __restrict__ hc, int ldh,
                                                               typename V2<R>::T* __restrict__ w, int64_t N,
                                                               double* __restrict__ partial,
                                                               const double* __restrict__ nrm0,
                                                               const double* __restrict__ nrm1) {
    __shared__ R hs[2 * 64];
    __shared__ double sh[4];
    const int rhs = blockIdx.y;
    if (!second_pass(nrm0, nrm1, rhs)) {
        if (partial && threadIdx.x == 0)
            partial[static_cast<int64_t>(rhs) * gridDim.x + blockIdx.x] =
                blockIdx.x == 0 ? nrm1[rhs] * nrm1[rhs] : 0.0;
        return;
    }
    for (int j = threadIdx.x; j < J; j += kRedBlock) {
        const double2 c = hc[static_cast<int64_t>(rhs) * ldh + j];
        hs[2 * j] = static_cast<R>(c.x);
        hs[2 * j + 1] = static_cast<R>(c.y);
    }
    __syncthreads();
    typename V2<R>::T* wr = w + static_cast<int64_t>(rhs) * N;
    double nrm[1] = {0.0};
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock) {
        typename V2<R>::T acc = wr[i];
        for (int j = 0; j < J; ++j) {
            const typename V2<R>::T v = V[static_cast<int64_t>(j) * vstride + static_cast<int64_t>(rhs) * N + i];
            const R hr = hs[2 * j], hi = hs[2 * j + 1];
            acc.x -= v.x * hr - v.y * hi;
            acc.y -= v.x * hi + v.y * hr;
        }
        wr[i] = acc;
        nrm[0] += static_cast<double>(acc.x) * acc.x + static_cast<double>(acc.y) * acc.y;
    }
    if (partial) {
        block_sum<1>(nrm, sh);
        if (threadIdx.x == 0) partial[static_cast<int64_t>(rhs) * gridDim.x + blockIdx.x] = nrm[0];
    }
}

template <typename R>
int cgs_update(const void* V, int64_t vstride, int J, const double2* d_hc, int ldh, void* w, int64_t N, int nrhs,
               double* d_partial, int max_blocks, double* d_nrm, hipStream_t s, const double* d_gate0,
               const double* d_gate1) {
    if (J > 64) return HELM27_EINVAL;
    unsigned nb = grid_for(N);
    if (d_nrm && nb > static_cast<unsigned>(max_blocks)) nb = max_blocks;
    hipLaunchKernelGGL(cgs_update_kernel<R>, dim3(nb, nrhs), dim3(kRedBlock), 0, s,
                       static_cast<const typename V2<R>::T*>(V), vstride, J, d_hc, ldh,
                       static_cast<typename V2<R>::T*>(w), N, d_nrm ? d_partial : nullptr, d_gate0, d_gate1);
    if (d_nrm)
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(nrhs), dim3(kRedBlock), 0, s, d_partial, static_cast<int>(nb),
                           d_nrm, 1);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int cgs_update<float>(const void*, int64_t, int, const double2*, int, void*, int64_t, int, double*, int,
                               double*, hipStream_t, const double*, const double*);
template int cgs_update<double>(const void*, int64_t, int, const double2*, int, void*, int64_t, int, double*, int,
                                double*, hipStream_t, const double*, const double*);

// out[rhs] = x[rhs] * f(nrm[rhs]): mode 0 -> 1/nrm (0 if nrm == 0), mode 1 -> nrm
template <typename Ri, typename Ro>
__global__ void scale_kernel(const typename V2<Ri>::T* __restrict__ x, typename V2<Ro>::T* __restrict__ out,
                             typename V2<Ro>::T* __restrict__ out2, int64_t N, const double* __restrict__ nrm,
                             int mode, const typename V2<Ro>::T* __restrict__ dinv,
                             typename V2<Ro>::T* __restrict__ yout) {
    const int rhs = blockIdx.y;
    const double n = nrm[rhs];
    const double f = mode == 0 ? (n > 0 ? 1.0 / n : 0.0) : n;
    const typename V2<Ri>::T* xr = x + static_cast<int64_t>(rhs) * N;
    typename V2<Ro>::T* orr = out + static_cast<int64_t>(rhs) * N;
    typename V2<Ro>::T* orr2 = out2 ? out2 + static_cast<int64_t>(rhs) * N : nullptr;
    typename V2<Ro>::T* yr = yout ? yout + static_cast<int64_t>(rhs) * N : nullptr;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock) {
        const typename V2<Ri>::T v = xr[i];
        typename V2<Ro>::T o;
        o.x = static_cast<Ro>(static_cast<double>(v.x) * f);
        o.y = static_cast<Ro>(static_cast<double>(v.y) * f);
        orr[i] = o;
        if (orr2) orr2[i] = o;
        if (yr) yr[i] = dmul(dinv[i], o);
    }
}

template <typename Ri, typename Ro>
int scale_by_norm(const void* x, void* out, int64_t N, int nrhs, const double* d_nrm, int mode, hipStream_t s,
                  void* out2, const void* dinv, void* yout) {
    using Vo = typename V2<Ro>::T;
    hipLaunchKernelGGL((scale_kernel<Ri, Ro>), dim3(grid_for(N), nrhs), dim3(kRedBlock), 0, s,
                       static_cast<const typename V2<Ri>::T*>(x), static_cast<Vo*>(out), static_cast<Vo*>(out2), N,
                       d_nrm, mode, static_cast<const Vo*>(dinv), dinv ? static_cast<Vo*>(yout) : nullptr);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int scale_by_norm<float, float>(const void*, void*, int64_t, int, const double*, int, hipStream_t, void*,
                                          const void*, void*);
template int scale_by_norm<double, double>(const void*, void*, int64_t, int, const double*, int, hipStream_t, void*,
                                          const void*, void*);
template int scale_by_norm<double, float>(const void*, void*, int64_t, int, const double*, int, hipStream_t, void*,
                                          const void*, void*);

// u64[rhs] += nrm[rhs] * e[rhs]  (refinement update, e in the inner precision)
template <typename R>
__global__ void refine_update_kernel(double2* __restrict__ u, const typename V2<R>::T* __restrict__ e, int64_t N,
                                     const double* __restrict__ nrm) {
    const int rhs = blockIdx.y;
    const double f = nrm[rhs];
    double2* ur = u + static_cast<int64_t>(rhs) * N;
    const typename V2<R>::T* er = e + static_cast<int64_t>(rhs) * N;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock) {
        const typename V2<R>::T v = er[i];
        double2 a = ur[i];
        a.x += f * static_cast<double>(v.x);
        a.y += f * static_cast<double>(v.y);
        ur[i] = a;
    }
}

template <typename R>
int refine_update(double2* u, const void* e, int64_t N, int nrhs, const double* d_nrm, hipStream_t s) {
    hipLaunchKernelGGL(refine_update_kernel<R>, dim3(grid_for(N), nrhs), dim3(kRedBlock), 0, s, u,
                       static_cast<const typename V2<R>::T*>(e), N, d_nrm);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int refine_update<float>(double2*, const void*, int64_t, int, const double*, hipStream_t);
template int refine_update<double>(double2*, const void*, int64_t, int, const double*, hipStream_t);

// x[rhs] (+)= sum_{j<k} V_j[rhs] * y[rhs][j]
template <typename R>
__global__ __launch_bounds__(kRedBlock) void combine_kernel(const typename V2<R>::T* __restrict__ V, int64_t vstride, int k,
                                                            const double2* __restrict__ y, int ldy,
                                                            typename V2<R>::T* __restrict__ x, int64_t N, int accumulate,
                                                            const typename V2<R>::T* __restrict__ dinv,
                                                            typename V2<R>::T* __restrict__ yout) {
    __shared__ R ys[2 * 64];
    const int rhs = blockIdx.y;
    for (int j = threadIdx.x; j < k; j += kRedBlock) {
        const double2 c = y[static_cast<int64_t>(rhs) * ldy + j];
        ys[2 * j] = static_cast<R>(c.x);
        ys[2 * j + 1] = static_cast<R>(c.y);
    }
    __syncthreads();
    typename V2<R>::T* xr = x + static_cast<int64_t>(rhs) * N;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock) {
        typename V2<R>::T acc;
        if (accumulate) {
            acc = xr[i];
        } else {
            acc.x = R(0);
            acc.y = R(0);
        }
        for (int j = 0; j < k; ++j) {
            const typename V2<R>::T v = V[static_cast<int64_t>(j) * vstride + static_cast<int64_t>(rhs) * N + i];
            const R yr = ys[2 * j], yi = ys[2 * j + 1];
            acc.x += v.x * yr - v.y * yi;
            acc.y += v.x * yi + v.y * yr;
        }
        xr[i] = acc;
        if (yout) yout[static_cast<int64_t>(rhs) * N + i] = dmul(dinv[i], acc);
    }
}

template <typename R>
int combine(const void* V, int64_t vstride, int k, const double2* d_y, int ldy, void* x, int64_t N, int nrhs,
            int accumulate, hipStream_t s, const void* dinv, void* yout) {
    using VT = typename V2<R>::T;
    if (k > 64) return HELM27_EINVAL;
    hipLaunchKernelGGL(combine_kernel<R>, dim3(grid_for(N), nrhs), dim3(kRedBlock), 0, s, static_cast<const VT*>(V),
                       vstride, k, d_y, ldy, static_cast<VT*>(x), N, accumulate, static_cast<const VT*>(dinv),
                       dinv ? static_cast<VT*>(yout) : nullptr);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int combine<float>(const void*, int64_t, int, const double2*, int, void*, int64_t, int, int, hipStream_t,
                            const void*, void*);
template int combine<double>(const void*, int64_t, int, const double2*, int, void*, int64_t, int, int, hipStream_t,
                             const void*, void*);

// x[rhs] += y[rhs]
template <typename R>
__global__ void axpy1_kernel(typename V2<R>::T* __restrict__ x, const typename V2<R>::T* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedBlock) {
        typename V2<R>::T a = x[i];
        const typename V2<R>::T b = y[i];
        a.x += b.x;
        a.y += b.y;
        x[i] = a;
    }
}

template <typename R>
int add_inplace(void* x, const void* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpy1_kernel<R>, dim3(grid_for(n)), dim3(kRedBlock), 0, s, static_cast<typename V2<R>::T*>(x),
                       static_cast<const typename V2<R>::T*>(y), n);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int add_inplace<float>(void*, const void*, int64_t, hipStream_t);
template int add_inplace<double>(void*, const void*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// GMRES bookkeeping in FP64, one thread per right-hand side.
// Layout per rhs: H [(m+1) x m] column-major (H[i + (m+1) j]), cs [m], sn [m]
// (complex), g [m+1] (complex).  hcol[rhs][0..j] holds the orthogonalisation
// coefficients of step j, nrm[rhs] = ||w|| = H(j+1, j).
__global__ void givens_kernel(int j, int m, int nrhs, const double2* __restrict__ hcol, int ldh,
                              const double* __restrict__ nrm, double2* __restrict__ H, double* __restrict__ cs,
                              double2* __restrict__ sn, double2* __restrict__ g, double* __restrict__ est) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double2* Hr = H + static_cast<int64_t>(r) * (m + 1) * m;
    double* c = cs + static_cast<int64_t>(r) * m;
    double2* s = sn + static_cast<int64_t>(r) * m;
    double2* gr = g + static_cast<int64_t>(r) * (m + 1);
    double2* col = Hr + static_cast<int64_t>(j) * (m + 1);
    const double2* hc = hcol + static_cast<int64_t>(r) * ldh;
    // previous rotations on the new column (entries 0..j of hcol, then
    // ||w||): [a; b] <- [c a + s b; -conj(s) a + c b].  Entry i + 1 enters
    // unrotated, entry i carries the previous rotation's second output, so only
    // the carry is a dependence; the loads are independent of it.
    double2 carry = hc[0];
    for (int i = 0; i < j; ++i) {
        const double2 a = carry, b = hc[i + 1];
        const double ci = c[i];
        const double2 si = s[i];
        double2 t;
        t.x = ci * a.x + (si.x * b.x - si.y * b.y);
        t.y = ci * a.y + (si.x * b.y + si.y * b.x);
        carry.x = -(si.x * a.x + si.y * a.y) + ci * b.x;
        carry.y = -(si.x * a.y - si.y * a.x) + ci * b.y;
        col[i] = t;
    }
    const double2 a = carry;
    double2 b;
    b.x = nrm[r];
    b.y = 0.0;
    const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
    const double rho = hypot(na, nb);
    double cj;
    double2 sj;
    if (na == 0.0) {
        cj = 0.0;
        sj.x = 1.0;
        sj.y = 0.0;
    } else {
        cj = na / rho;
        // s = (a / |a|) conj(b) / rho
        const double ax = a.x / na, ay = a.y / na;
        sj.x = (ax * b.x + ay * b.y) / rho;
        sj.y = (ay * b.x - ax * b.y) / rho;
    }
    c[j] = cj;
    s[j] = sj;
    double2 rj;
    rj.x = cj * a.x + (sj.x * b.x - sj.y * b.y);
    rj.y = cj * a.y + (sj.x * b.y + sj.y * b.x);
    col[j] = rj;
    col[j + 1].x = 0.0;
    col[j + 1].y = 0.0;
    const double2 gj = gr[j];
    double2 g1;
    g1.x = -(sj.x * gj.x + sj.y * gj.y);
    g1.y = -(sj.x * gj.y - sj.y * gj.x);
    gr[j + 1] = g1;
    gr[j].x = cj * gj.x;
    gr[j].y = cj * gj.y;
    est[r] = hypot(g1.x, g1.y);
}

int givens_step(int j, int m, int nrhs, const double2* hcol, int ldh, const double* nrm, double2* H, double* cs,
                double2* sn, double2* g, double* est, hipStream_t s) {
    hipLaunchKernelGGL(givens_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, s, j, m, nrhs, hcol, ldh, nrm, H, cs, sn, g,
                       est);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

// g[rhs][0] = beta[rhs], rest 0
__global__ void ginit_kernel(double2* __restrict__ g, int m, int nrhs, const double* __restrict__ beta) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double2* gr = g + static_cast<int64_t>(r) * (m + 1);
    for (int i = 0; i <= m; ++i) {
        gr[i].x = 0.0;
        gr[i].y = 0.0;
    }
    gr[0].x = beta[r];
}

int givens_init(double2* g, int m, int nrhs, const double* beta, hipStream_t s) {
    hipLaunchKernelGGL(ginit_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, s, g, m, nrhs, beta);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

// y[rhs][0..k) = R_k^{-1} g_k (upper-triangular back substitution)
__global__ void upper_solve_kernel(int k, int m, int nrhs, const double2* __restrict__ H, const double2* __restrict__ g,
                                   double2* __restrict__ y, int ldy) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    const double2* Hr = H + static_cast<int64_t>(r) * (m + 1) * m;
    const double2* gr = g + static_cast<int64_t>(r) * (m + 1);
    double2* yr = y + static_cast<int64_t>(r) * ldy;
    for (int i = k - 1; i >= 0; --i) {
        double sx = gr[i].x, sy = gr[i].y;
        for (int jj = i + 1; jj < k; ++jj) {
            const double2 h = Hr[i + static_cast<int64_t>(jj) * (m + 1)];
            const double2 v = yr[jj];
            sx -= h.x * v.x - h.y * v.y;
            sy -= h.x * v.y + h.y * v.x;
        }
        const double2 d = Hr[i + static_cast<int64_t>(i) * (m + 1)];
        const double dd = d.x * d.x + d.y * d.y;
        double2 o;
        if (dd > 0) {
            o.x = (sx * d.x + sy * d.y) / dd;
            o.y = (sy * d.x - sx * d.y) / dd;
        } else {
            o.x = 0.0;
            o.y = 0.0;
        }
        yr[i] = o;
    }
}

int upper_solve(int k, int m, int nrhs, const double2* H, const double2* g, double2* y, int ldy, hipStream_t s) {
    hipLaunchKernelGGL(upper_solve_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, s, k, m, nrhs, H, g, y, ldy);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

// ---------------------------------------------------------------------------
// Multigrid transfers between a grid (nx, ny, nz) and its coarse grid
// ((nx+1)/2, ...): coarse node i sits on fine node 2i.  Full weighting
// (1/4, 1/2, 1/4 per axis, fine nodes outside the grid count as zero) and its
// adjoint up to a factor 8, trilinear interpolation.
constexpr int kXferRows = 4;   // y rows per transfer block (one wavefront each)

template <typename R>
__global__ __launch_bounds__(64 * kXferRows) void restrict_kernel(const typename V2<R>::T* __restrict__ f, int nx,
                                                                 int ny, int nz, typename V2<R>::T* __restrict__ c,
                                                                 int cx, int cy, int cz, int nrhs,
                                                                 const typename V2<R>::T* __restrict__ dinv,
                                                                 typename V2<R>::T* __restrict__ yout) {
    // one coarse node per thread: x from the block's 64-wide strip, y from the
    // block's rows, (z, rhs) from the grid (no integer division per thread).
    // The 27 fine loads use clamped indices (weight 0 outside the grid), so
    // every one of them is issued before the first is used.
    using V = typename V2<R>::T;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * kXferRows + (threadIdx.x >> 6);
    const int k = blockIdx.z % cz, rhs = blockIdx.z / cz;
    if (i >= cx || j >= cy) return;
    const int64_t Nf = static_cast<int64_t>(nx) * ny * nz;
    const V* fr = f + static_cast<int64_t>(rhs) * Nf;
    int xs[3], ys[3], zs[3];
    R wx[3], wy[3], wz[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R wd = d == 1 ? R(0.5) : R(0.25);
        const int x = 2 * i + d - 1, y = 2 * j + d - 1, z = 2 * k + d - 1;
        wx[d] = x >= 0 && x < nx ? wd : R(0);
        wy[d] = y >= 0 && y < ny ? wd : R(0);
        wz[d] = z >= 0 && z < nz ? wd : R(0);
        xs[d] = min(max(x, 0), nx - 1);
        ys[d] = min(max(y, 0), ny - 1);
        zs[d] = min(max(z, 0), nz - 1);
    }
    V v[27];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const V* row = fr + (static_cast<int64_t>(zs[a]) * ny + ys[b]) * nx;
#pragma unroll
            for (int d = 0; d < 3; ++d) v[(a * 3 + b) * 3 + d] = row[xs[d]];
        }
    R sx = 0, sy = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const R wab = wz[a] * wy[b];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const R w = wab * wx[d];
                sx += w * v[(a * 3 + b) * 3 + d].x;
                sy += w * v[(a * 3 + b) * 3 + d].y;
            }
        }
    V o;
    o.x = sx;
    o.y = sy;
    const int64_t pc = (static_cast<int64_t>(k) * cy + j) * cx + i;
    c[static_cast<int64_t>(rhs) * cx * cy * cz + pc] = o;
    if (yout) yout[static_cast<int64_t>(rhs) * cx * cy * cz + pc] = dmul(dinv[pc], o);   // first coarse sweep
}

template <typename R>
__global__ __launch_bounds__(64 * kXferRows) void prolong_add_kernel(const typename V2<R>::T* __restrict__ c, int cx,
                                                                    int cy, int cz, typename V2<R>::T* __restrict__ f,
                                                                    int nx, int ny, int nz, int nrhs) {
    // trilinear interpolation of the coarse correction, added to the fine
    // iterate.  One thread per fine (x, y) and pair of fine planes 2p, 2p + 1,
    // which share coarse plane p: x from the block's strip, y from the block's
    // rows, (p, rhs) from the grid.  Per axis an even node takes one coarse
    // node (weight 1), an odd node two (1/2 each); the second node's index is
    // clamped and its weight is 0 where it is not used, so all eight coarse
    // loads and both fine loads are issued at once.
    using V = typename V2<R>::T;
    const int ncp = (nz + 1) / 2;   // plane pairs
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * kXferRows + (threadIdx.x >> 6);
    const int zp = blockIdx.z % ncp, rhs = blockIdx.z / ncp;
    if (x >= nx || y >= ny) return;
    const V* cr = c + static_cast<int64_t>(rhs) * cx * cy * cz;
    const int x0 = x >> 1, y0 = y >> 1;
    const int x1 = min(x0 + 1, cx - 1), y1 = min(y0 + 1, cy - 1), z1 = min(zp + 1, cz - 1);
    const R hx = (x & 1) && x0 + 1 < cx ? R(0.5) : R(0), hy = (y & 1) && y0 + 1 < cy ? R(0.5) : R(0);
    const R hz = zp + 1 < cz ? R(0.5) : R(0);   // the odd plane's upper coarse plane
    const R gx = (x & 1) ? R(0.5) : R(1), gy = (y & 1) ? R(0.5) : R(1);
    const bool odd = 2 * zp + 1 < nz;
    V* fe = f + static_cast<int64_t>(rhs) * nx * ny * nz + (static_cast<int64_t>(2 * zp) * ny + y) * nx + x;
    V* fo = odd ? fe + static_cast<int64_t>(nx) * ny : fe;
    const V* r00 = cr + (static_cast<int64_t>(zp) * cy + y0) * cx;
    const V* r01 = cr + (static_cast<int64_t>(zp) * cy + y1) * cx;
    const V* r10 = cr + (static_cast<int64_t>(z1) * cy + y0) * cx;
    const V* r11 = cr + (static_cast<int64_t>(z1) * cy + y1) * cx;
    const V a0 = r00[x0], a1 = r00[x1], b0 = r01[x0], b1 = r01[x1];
    const V c0 = r10[x0], c1 = r10[x1], d0 = r11[x0], d1 = r11[x1];
    V oe = *fe, oo = *fo;
    // interpolated in x and y on coarse planes zp (P) and zp + 1 (Q)
    const R px = gy * (gx * a0.x + hx * a1.x) + hy * (gx * b0.x + hx * b1.x);
    const R py = gy * (gx * a0.y + hx * a1.y) + hy * (gx * b0.y + hx * b1.y);
    const R qx = gy * (gx * c0.x + hx * c1.x) + hy * (gx * d0.x + hx * d1.x);
    const R qy = gy * (gx * c0.y + hx * c1.y) + hy * (gx * d0.y + hx * d1.y);
    oe.x += px;
    oe.y += py;
    *fe = oe;
    if (odd) {
        oo.x += R(0.5) * px + hz * qx;
        oo.y += R(0.5) * py + hz * qy;
        *fo = oo;
    }
}

template <typename R>
int mg_restrict(const void* f, int nx, int ny, int nz, void* c, int cx, int cy, int cz, int nrhs, hipStream_t s,
                const void* dinv, void* yout) {
    using V = typename V2<R>::T;
    if (static_cast<int64_t>(cx) * cy * cz * nrhs <= 0) return HELM27_OK;
    if (cy > 65535 || cz > 65535) return HELM27_EINVAL;
    const int per = 65535 / cz;   // right-hand sides per launch (grid z = cz * count)
    const int64_t Nf = static_cast<int64_t>(nx) * ny * nz, Nc = static_cast<int64_t>(cx) * cy * cz;
    for (int r0 = 0; r0 < nrhs; r0 += per) {
        const int n = nrhs - r0 < per ? nrhs - r0 : per;
        H27_CHECK_HIP(launch(restrict_kernel<R>, dim3((cx + 63) / 64, (cy + kXferRows - 1) / kXferRows, cz * n),
                             dim3(64 * kXferRows), 0, s,
                             static_cast<const V*>(f) + r0 * Nf, nx, ny, nz, static_cast<V*>(c) + r0 * Nc, cx, cy, cz,
                             n, static_cast<const V*>(dinv), dinv ? static_cast<V*>(yout) + r0 * Nc : nullptr));
    }
    return HELM27_OK;
}
template <typename R>
int mg_prolong_add(const void* c, int cx, int cy, int cz, void* f, int nx, int ny, int nz, int nrhs, hipStream_t s) {
    using V = typename V2<R>::T;
    if (static_cast<int64_t>(nx) * ny * nz * nrhs <= 0) return HELM27_OK;
    if (ny > 65535 || nz > 65535) return HELM27_EINVAL;
    const int per = 65535 / nz;   // right-hand sides per launch (grid z = nz * count)
    const int64_t Nf = static_cast<int64_t>(nx) * ny * nz, Nc = static_cast<int64_t>(cx) * cy * cz;
    for (int r0 = 0; r0 < nrhs; r0 += per) {
        const int n = nrhs - r0 < per ? nrhs - r0 : per;
        H27_CHECK_HIP(launch(prolong_add_kernel<R>,
                             dim3((nx + 63) / 64, (ny + kXferRows - 1) / kXferRows, (nz + 1) / 2 * n),
                             dim3(64 * kXferRows), 0, s,
                             static_cast<const V*>(c) + r0 * Nc, cx, cy, cz, static_cast<V*>(f) + r0 * Nf, nx, ny,
                             nz, n));
    }
    return HELM27_OK;
}
template int mg_restrict<float>(const void*, int, int, int, void*, int, int, int, int, hipStream_t, const void*, void*);
template int mg_restrict<double>(const void*, int, int, int, void*, int, int, int, int, hipStream_t, const void*,
                                 void*);
template int mg_prolong_add<float>(const void*, int, int, int, void*, int, int, int, int, hipStream_t);
template int mg_prolong_add<double>(const void*, int, int, int, void*, int, int, int, int, hipStream_t);

// c_coarse[k][j][i] = c_fine[2k][2j][2i] (velocity injected to the coarse grid)
__global__ void inject_velocity_kernel(const float* __restrict__ f, int nx, int ny, float* __restrict__ c, int cx, int cy,
                                       int cz) {
    const int64_t Nc = static_cast<int64_t>(cx) * cy * cz;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < Nc;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(t % cx), j = static_cast<int>((t / cx) % cy), k = static_cast<int>(t / (static_cast<int64_t>(cx) * cy));
        c[t] = f[2 * i + static_cast<int64_t>(nx) * (2 * j + static_cast<int64_t>(ny) * 2 * k)];
    }
}

int inject_velocity(const float* f, int nx, int ny, float* c, int cx, int cy, int cz, hipStream_t s) {
    const int64_t total = static_cast<int64_t>(cx) * cy * cz;
    hipLaunchKernelGGL(inject_velocity_kernel, dim3(grid_for(total, 1)), dim3(kRedBlock), 0, s, f, nx, ny, c, cx, cy, cz);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

}  // namespace h27
