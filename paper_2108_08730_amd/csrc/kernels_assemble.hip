// Assembly kernels: per-point table index, stored 27-coefficient operator,
// "GAm" neighbourhood-averaged weights, and the stored-coefficient apply.
//
// This file is compiled with -ffp-contract=off: the table index must be the
// same binary64 result as the same formula evaluated anywhere else.
#include "stencil.h"

#include <climits>
#include <cmath>
#include <cstring>

namespace h27 {

// idx = clamp(floor((v - v_min)/dv + 1/2), 0, n_g - 1) with v = c/(f h) on the
// G axis and v = (f h)/c on the 1/G axis (paper Sec. 3.1: every row picks the
// table entry of its local G = c/(f h); nearest entry, ties upwards).  counts[0] += clamped points, counts[1] += invalid velocities,
// counts[2] / counts[3] = min / max bit pattern of the valid velocities (the
// bits of positive floats order like the values; the caller initialises them
// to +inf and 0).
// One point: its table index, and the running clamp / invalid counts and
// velocity range of the calling thread.
__device__ __forceinline__ uint16_t index_point(float cv, double fh, double gmin, double dg, int n_g, int invg,
                                                unsigned long long& ncl, unsigned long long& nbad, float& vmin,
                                                float& vmax) {
    const double top = static_cast<double>(n_g - 1);
    if (!(cv > 0.0f) || !isfinite(cv)) {
        ++nbad;
    } else {
        vmin = fminf(vmin, cv);
        vmax = fmaxf(vmax, cv);
    }
    const double G = invg ? fh / static_cast<double>(cv) : static_cast<double>(cv) / fh;
    const double t = (G - gmin) / dg;
    const double raw = floor(t + 0.5);
    int k;
    if (!(raw >= 0.0)) {
        k = 0;
        ++ncl;
    } else if (raw > top) {
        k = n_g - 1;
        ++ncl;
    } else {
        k = static_cast<int>(raw);
    }
    return static_cast<uint16_t>(k);
}

__global__ void select_index_kernel(const float* __restrict__ c, uint16_t* __restrict__ idx, int64_t N,
                                    double fh, double gmin, double dg, int n_g, int invg,
                                    unsigned long long* __restrict__ counts) {
    __shared__ unsigned long long red[2][kBlock / 64];
    __shared__ float rmm[2][kBlock / 64];
    unsigned long long ncl = 0, nbad = 0;
    float vmin = __builtin_inff(), vmax = 0.0f;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        idx[i] = index_point(c[i], fh, gmin, dg, n_g, invg, ncl, nbad, vmin, vmax);
    // wavefront reduction, then one atomic per block
    for (int off = 32; off > 0; off >>= 1) {
        ncl += __shfl_down(ncl, off, 64);
        nbad += __shfl_down(nbad, off, 64);
        vmin = fminf(vmin, __shfl_down(vmin, off, 64));
        vmax = fmaxf(vmax, __shfl_down(vmax, off, 64));
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        red[0][w] = ncl;
        red[1][w] = nbad;
        rmm[0][w] = vmin;
        rmm[1][w] = vmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        float mn = __builtin_inff(), mx = 0.0f;
        for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) {
            a += red[0][k];
            b += red[1][k];
            mn = fminf(mn, rmm[0][k]);
            mx = fmaxf(mx, rmm[1][k]);
        }
        if (a) atomicAdd(counts, a);
        if (b) atomicAdd(counts + 1, b);
        // min / max only change monotonically, so an earlier value read
        // without the atomic safely rules out most updates (thousands of
        // blocks contending for one address otherwise serialise)
        const unsigned long long lo = __float_as_uint(mn), hi = __float_as_uint(mx);
        if (lo < __hip_atomic_load(counts + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(counts + 2, lo);
        if (hi > __hip_atomic_load(counts + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(counts + 3, hi);
    }
}

// ---------------------------------------------------------------------------
// Index selection that allocates nothing (helm27_select_index_noalloc): each
// block of the first kernel handles a fixed range of kNaPerBlock points and
// writes its counts and velocity range to its own record of a file-scope
// device array; the second kernel reduces the records in a fixed order into
// the last record.  Every record a launch reads was written by that launch,
// so nothing needs clearing between calls.
struct NaRecord {
    unsigned long long ncl, nbad, minbits, maxbits;
};
constexpr int kNaBlocks = 4096;                  // partial records (blocks) at most
constexpr int64_t kNaPerBlock = 65536;           // points per block
constexpr int64_t kNaMaxPoints = kNaBlocks * kNaPerBlock;   // 268,435,456 points
// kNaBlocks partial records + the reduced record: 131 KB per device
static __device__ __align__(256) NaRecord scratch[kNaBlocks + 1];

__device__ __forceinline__ void block_reduce_record(unsigned long long ncl, unsigned long long nbad, float vmin,
                                                    float vmax, NaRecord* out) {
    __shared__ unsigned long long red[2][kBlock / 64];
    __shared__ float rmm[2][kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        ncl += __shfl_down(ncl, off, 64);
        nbad += __shfl_down(nbad, off, 64);
        vmin = fminf(vmin, __shfl_down(vmin, off, 64));
        vmax = fmaxf(vmax, __shfl_down(vmax, off, 64));
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        red[0][w] = ncl;
        red[1][w] = nbad;
        rmm[0][w] = vmin;
        rmm[1][w] = vmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        NaRecord r{0, 0, 0, 0};
        float mn = __builtin_inff(), mx = 0.0f;
        for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) {
            r.ncl += red[0][k];
            r.nbad += red[1][k];
            mn = fminf(mn, rmm[0][k]);
            mx = fmaxf(mx, rmm[1][k]);
        }
        r.minbits = __float_as_uint(mn);
        r.maxbits = __float_as_uint(mx);
        *out = r;
    }
}

__global__ __launch_bounds__(kBlock) void select_index_blocks_kernel(const float* __restrict__ c,
                                                                     uint16_t* __restrict__ idx, int64_t N, double fh,
                                                                     double gmin, double dg, int n_g, int invg,
                                                                     NaRecord* __restrict__ rec) {
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kNaPerBlock;
    const int64_t i1 = i0 + kNaPerBlock < N ? i0 + kNaPerBlock : N;
    unsigned long long ncl = 0, nbad = 0;
    float vmin = __builtin_inff(), vmax = 0.0f;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock)
        idx[i] = index_point(c[i], fh, gmin, dg, n_g, invg, ncl, nbad, vmin, vmax);
    block_reduce_record(ncl, nbad, vmin, vmax, rec + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void reduce_records_kernel(const NaRecord* __restrict__ rec, int nrec,
                                                                NaRecord* __restrict__ out) {
    unsigned long long ncl = 0, nbad = 0;
    float vmin = __builtin_inff(), vmax = 0.0f;
    for (int k = threadIdx.x; k < nrec; k += kBlock) {
        const NaRecord r = rec[k];
        ncl += r.ncl;
        nbad += r.nbad;
        vmin = fminf(vmin, __uint_as_float(static_cast<unsigned>(r.minbits)));
        vmax = fmaxf(vmax, __uint_as_float(static_cast<unsigned>(r.maxbits)));
    }
    block_reduce_record(ncl, nbad, vmin, vmax, out);
}

// device address of this device's scratch array (looked up once per device,
// with that device current)
static int scratch_address(int device, NaRecord** out) {
    static std::mutex mu;
    static std::vector<NaRecord*> ptrs;
    std::lock_guard<std::mutex> lk(mu);
    if (device < 0) return HELM27_EINVAL;
    if (static_cast<size_t>(device) >= ptrs.size()) ptrs.resize(device + 1, nullptr);
    if (!ptrs[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            std::fprintf(stderr, "helm27: hipGetSymbolAddress(scratch) failed on device %d: %s\n", device,
                         hipGetErrorString(e));
            return HELM27_EDEVICE;
        }
        ptrs[device] = static_cast<NaRecord*>(p);
    }
    *out = ptrs[device];
    return HELM27_OK;
}

int noalloc_init(int device) {
    NaRecord* p = nullptr;
    return scratch_address(device, &p);
}

int launch_select_index(const float* c, uint16_t* idx, int64_t N, double fh, double gmin, double dg,
                        int n_g, int invg, unsigned long long* d_counts, hipStream_t s) {
    int64_t blocks = (N + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(select_index_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, c, idx, N,
                       fh, gmin, dg, n_g, invg, d_counts);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

// ---------------------------------------------------------------------------
// 27 coefficients of one row, written to coef_at(i, s) (s = (dz+1)*9 +
// (dy+1)*3 + (dx+1)); zero where the neighbour lies outside the grid.
template <typename R>
__global__ void fill_stored_kernel(GridData<R> g, typename V2<R>::T* __restrict__ coef) {
    const int64_t N = g.N;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(i % g.nx);
        const int y = static_cast<int>((i / g.nx) % g.ny);
        const int z = static_cast<int>(i / g.plane);
        const AxisNode<R>* nodes[3] = {g.ax + x, g.ay + y, g.az + z};
        const int pos[3] = {x, y, z};
        const int ext[3] = {g.nx, g.ny, g.nz};
        Cx<R> T[3][3], X[3][3], U[3][3];
        for (int a = 0; a < 3; ++a) {
            const AxisNode<R> n = *nodes[a];
            const Cx<R> tm = mk(n.tm_re, n.tm_im), tp = mk(n.tp_re, n.tp_im);
            T[a][0] = tm;
            T[a][1] = -(tm + tp);
            T[a][2] = tp;
            X[a][0] = zero<R>();
            X[a][1] = mk(n.xi_re, n.xi_im);
            X[a][2] = zero<R>();
            U[a][0] = mk(n.um_re, n.um_im);
            U[a][1] = zero<R>();
            U[a][2] = mk(n.up_re, n.up_im);
        }
        EntryCoef<R> E;
        if (g.rowcoef) E = g.rowcoef[i];
        else E = g.entry[g.fixed ? 0 : g.idx[i]];
        const R cv = static_cast<R>(g.c[i]);
        const R kap = g.omega2 / (cv * cv);
        const Cx<R> kc = mk(kap * g.shift_re, kap * g.shift_im);
        const R sig = g.inv_h2;
        for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy)
                for (int dx = 0; dx < 3; ++dx) {
                    const int s = dz * 9 + dy * 3 + dx;
                    const int d[3] = {dx, dy, dz};
                    bool inside = true;
                    for (int a = 0; a < 3; ++a) {
                        const int p = pos[a] + d[a] - 1;
                        inside = inside && p >= 0 && p < ext[a];
                    }
                    Cx<R> val = zero<R>();
                    if (inside) {
                        const Cx<R> tx = T[0][dx], ty = T[1][dy], tz = T[2][dz];
                        const Cx<R> xx = X[0][dx], xy = X[1][dy], xz = X[2][dz];
                        const Cx<R> ux = U[0][dx], uy = U[1][dy], uz = U[2][dz];
                        Cx<R> stiff = tx * xy * xz + xx * ty * xz + xx * xy * tz;
                        stiff = stiff + E.beta2 * (tx * ty * xz + tx * xy * tz + xx * ty * tz);
                        stiff = stiff + E.beta3 * (tx * ty * tz);
                        Cx<R> mass = E.m0 * (xx * xy * xz);
                        mass = mass + (R(2) * E.m1) * (ux * xy * xz + xx * uy * xz + xx * xy * uz);
                        mass = mass + (R(4) * E.m2) * (ux * uy * xz + ux * xy * uz + xx * uy * uz);
                        mass = mass + (R(8) * E.m3) * (ux * uy * uz);
                        if (g.mass_a) {
                            // first mass form: the neighbour's own bulk modulus
                            const int64_t j = i + (dx - 1) + (dy - 1) * static_cast<int64_t>(g.nx) +
                                              (dz - 1) * g.plane;
                            const R cj = static_cast<R>(g.c[j]);
                            const R kj = g.omega2 / (cj * cj);
                            val = sig * stiff + mk(kj * g.shift_re, kj * g.shift_im) * mass;
                        } else {
                            val = sig * stiff + kc * mass;
                        }
                    }
                    st<R>(coef + coef_at(i, s), val);
                }
    }
}

template <typename R>
static GridData<R> make_grid_data(const GridOp& g, double shift_re, double shift_im);

template <>
GridData<float> make_grid_data<float>(const GridOp& g, double shift_re, double shift_im) {
    GridData<float> d{};
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.plane = static_cast<int64_t>(g.nx) * g.ny;
    d.N = g.N;
    d.c = g.d_c; d.idx = g.d_idx; d.entry = g.d_entry_f; d.rowcoef = g.d_row_f; d.fixed = g.fixed;
    d.ax = g.d_ax_f[0]; d.ay = g.d_ax_f[1]; d.az = g.d_ax_f[2];
    d.omega2 = static_cast<float>(g.omega * g.omega);
    d.inv_h2 = static_cast<float>(1.0 / (g.h * g.h));
    // mass factor = requested shift x the medium's attenuation factor
    d.shift_re = static_cast<float>(shift_re * g.att_re - shift_im * g.att_im);
    d.shift_im = static_cast<float>(shift_re * g.att_im + shift_im * g.att_re);
    d.mass_a = g.mass_a;
    d.zlo = g.zp_lo;
    d.zhi = g.zp_hi;
    return d;
}

template <>
GridData<double> make_grid_data<double>(const GridOp& g, double shift_re, double shift_im) {
    GridData<double> d{};
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.plane = static_cast<int64_t>(g.nx) * g.ny;
    d.N = g.N;
    d.c = g.d_c; d.idx = g.d_idx; d.entry = g.d_entry_d; d.rowcoef = g.d_row_d; d.fixed = g.fixed;
    d.ax = g.d_ax_d[0]; d.ay = g.d_ax_d[1]; d.az = g.d_ax_d[2];
    d.omega2 = g.omega * g.omega;
    d.inv_h2 = 1.0 / (g.h * g.h);
    d.shift_re = shift_re * g.att_re - shift_im * g.att_im;
    d.shift_im = shift_re * g.att_im + shift_im * g.att_re;
    d.mass_a = g.mass_a;
    d.zlo = g.zp_lo;
    d.zhi = g.zp_hi;
    return d;
}

template <typename R>
int launch_fill_stored(const GridOp& g, void* coef, double shift_re, double shift_im, hipStream_t s) {
    GridData<R> d = make_grid_data<R>(g, shift_re, shift_im);
    int64_t blocks = (g.N + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(fill_stored_kernel<R>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, d,
                       static_cast<typename V2<R>::T*>(coef));
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int launch_fill_stored<float>(const GridOp&, void*, double, double, hipStream_t);
template int launch_fill_stored<double>(const GridOp&, void*, double, double, hipStream_t);

// ---------------------------------------------------------------------------
// Stored-coefficient apply: y_i = sum_s A_is u[i + off_s].  One point per
// thread, blocks in XCD-contiguous order.  The 27 coefficients of a row are
// streamed once (coalesced 64-row blocks, non-temporal so they do not evict u
// from L2) and reused for every right-hand side; u neighbours come through
// the caches; y is written non-temporally.
template <typename R>
__global__ __launch_bounds__(kBlock) void apply_stored_kernel(GridData<R> g, const typename V2<R>::T* __restrict__ coef,
                                                              const typename V2<R>::T* __restrict__ u,
                                                              typename V2<R>::T* __restrict__ y, int nrhs) {
    const int64_t N = g.N;
    const int64_t i = xcd_block() * kBlock + threadIdx.x;
    if (i < N) {
        const int x = static_cast<int>(i % g.nx);
        const int yy = static_cast<int>((i / g.nx) % g.ny);
        const int z = static_cast<int>(i / g.plane);
        Cx<R> cf[27];
#pragma unroll
        for (int s = 0; s < 27; ++s) cf[s] = ld_nt<R>(coef + coef_at(i, s));
        const bool xm = x > 0, xp = x < g.nx - 1, ym = yy > 0, yp = yy < g.ny - 1, zm = z > 0, zp = z < g.nz - 1;
        for (int r = 0; r < nrhs; ++r) {
            const typename V2<R>::T* ur = u + static_cast<int64_t>(r) * N;
            Cx<R> acc = zero<R>();
#pragma unroll
            for (int s = 0; s < 27; ++s) {
                const int dz = s / 9 - 1, dy = (s / 3) % 3 - 1, dx = s % 3 - 1;
                const bool ok = (dx < 0 ? xm : (dx > 0 ? xp : true)) && (dy < 0 ? ym : (dy > 0 ? yp : true)) &&
                                (dz < 0 ? zm : (dz > 0 ? zp : true));
                if (ok) cmac(acc, cf[s], ld<R>(ur + i + dx + static_cast<int64_t>(g.nx) * dy + g.plane * dz));
            }
            st_nt<R>(y + static_cast<int64_t>(r) * N + i, acc);
        }
    }
}

template <typename R>
int launch_apply_stored(const GridOp& g, const void* coef, const void* u, void* y, int nrhs, hipStream_t s) {
    GridData<R> d = make_grid_data<R>(g, 1.0, 0.0);
    const int64_t blocks = (g.N + kBlock - 1) / kBlock;   // one point per thread
    if (blocks > INT_MAX) return HELM27_EINVAL;
    hipLaunchKernelGGL(apply_stored_kernel<R>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, d,
                       static_cast<const typename V2<R>::T*>(coef), static_cast<const typename V2<R>::T*>(u),
                       static_cast<typename V2<R>::T*>(y), nrhs);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int launch_apply_stored<float>(const GridOp&, const void*, const void*, void*, int, hipStream_t);
template int launch_apply_stored<double>(const GridOp&, const void*, const void*, void*, int, hipStream_t);

// Transposed stored-coefficient apply: y_i = sum_s A[i + off_s][i] u[i + off_s]
// = sum_s A_{j, 26 - s} u[j] with j = i + off_s (the entry of row j
// towards i sits at the opposite offset), or with b: y = b - A^T u.  The
// coefficients are read at the neighbour's index, as coalesced as u.  Block
// order and caching as the stored apply.
template <typename R>
__global__ __launch_bounds__(kBlock) void apply_stored_t_kernel(GridData<R> g,
                                                                const typename V2<R>::T* __restrict__ coef,
                                                                const typename V2<R>::T* __restrict__ u,
                                                                const typename V2<R>::T* __restrict__ b,
                                                                typename V2<R>::T* __restrict__ y, int nrhs) {
    const int64_t N = g.N;
    const int64_t i = xcd_block() * kBlock + threadIdx.x;
    if (i < N) {
        const int x = static_cast<int>(i % g.nx);
        const int yy = static_cast<int>((i / g.nx) % g.ny);
        const int z = static_cast<int>(i / g.plane);
        const bool xm = x > 0, xp = x < g.nx - 1, ym = yy > 0, yp = yy < g.ny - 1, zm = z > 0, zp = z < g.nz - 1;
        for (int r = 0; r < nrhs; ++r) {
            const typename V2<R>::T* ur = u + static_cast<int64_t>(r) * N;
            Cx<R> acc = zero<R>();
#pragma unroll
            for (int s = 0; s < 27; ++s) {
                const int dz = s / 9 - 1, dy = (s / 3) % 3 - 1, dx = s % 3 - 1;
                const bool ok = (dx < 0 ? xm : (dx > 0 ? xp : true)) && (dy < 0 ? ym : (dy > 0 ? yp : true)) &&
                                (dz < 0 ? zm : (dz > 0 ? zp : true));
                if (ok) {
                    const int64_t j = i + dx + static_cast<int64_t>(g.nx) * dy + g.plane * dz;
                    cmac(acc, ld_nt<R>(coef + coef_at(j, 26 - s)), ld<R>(ur + j));
                }
            }
            if (b) acc = ld_nt<R>(b + static_cast<int64_t>(r) * N + i) - acc;
            st_nt<R>(y + static_cast<int64_t>(r) * N + i, acc);
        }
    }
}

template <typename R>
int launch_apply_stored_t(const GridOp& g, const void* coef, const void* u, void* y, const void* b, int nrhs,
                          hipStream_t s) {
    GridData<R> d = make_grid_data<R>(g, 1.0, 0.0);
    const int64_t blocks = (g.N + kBlock - 1) / kBlock;   // one point per thread
    if (blocks > INT_MAX) return HELM27_EINVAL;
    hipLaunchKernelGGL(apply_stored_t_kernel<R>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, d,
                       static_cast<const typename V2<R>::T*>(coef), static_cast<const typename V2<R>::T*>(u),
                       static_cast<const typename V2<R>::T*>(b), static_cast<typename V2<R>::T*>(y), nrhs);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int launch_apply_stored_t<float>(const GridOp&, const void*, const void*, void*, const void*, int,
                                          hipStream_t);
template int launch_apply_stored_t<double>(const GridOp&, const void*, const void*, void*, const void*, int,
                                           hipStream_t);

// ---------------------------------------------------------------------------
// "GAm": every row takes the mean of the table entries of its in-grid stencil
// points (paper Sec. 3.1).  The entry coefficients are linear in the weights,
// so averaging them equals deriving them from the averaged weights.
template <typename R>
__global__ void gam_average_kernel(GridData<R> g, EntryCoef<R>* __restrict__ out) {
    const int64_t N = g.N;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(i % g.nx);
        const int y = static_cast<int>((i / g.nx) % g.ny);
        const int z = static_cast<int>(i / g.plane);
        R acc[12];
        for (int k = 0; k < 12; ++k) acc[k] = R(0);
        int cnt = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx, yy = y + dy, zz = z + dz;
                    if (xx < 0 || xx >= g.nx || yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz) continue;
                    const int64_t j = i + dx + static_cast<int64_t>(g.nx) * dy + g.plane * dz;
                    const EntryCoef<R> E = g.entry[g.idx[j]];
                    const R* e = &E.s0;
                    for (int k = 0; k < 12; ++k) acc[k] += e[k];
                    ++cnt;
                }
        EntryCoef<R> o;
        R* op = &o.s0;
        for (int k = 0; k < 12; ++k) op[k] = acc[k] / static_cast<R>(cnt);
        out[i] = o;
    }
}

template <typename R>
int launch_gam_average(const GridOp& g, EntryCoef<R>* rowcoef, hipStream_t s) {
    GridData<R> d = make_grid_data<R>(g, 1.0, 0.0);
    d.rowcoef = nullptr;
    int64_t blocks = (g.N + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(gam_average_kernel<R>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, d, rowcoef);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}
template int launch_gam_average<float>(const GridOp&, EntryCoef<float>*, hipStream_t);
template int launch_gam_average<double>(const GridOp&, EntryCoef<double>*, hipStream_t);

}  // namespace h27

// a device pointer on `device` (host, managed-elsewhere or foreign pointers are refused)
static bool device_pointer_on(const void* p, int device) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice && at.device == device;
}

extern "C" int helm27_select_index_noalloc(helm27_ctx* ctx, const helm27_table* t, const float* vel, int64_t n,
                                           double h, double freq, uint16_t* idx, helm27_index_stats* stats,
                                           void* stream) {
    using namespace h27;
    if (!ctx || !t || !vel || !idx || t->n_g < 1 || !(h > 0.0) || !(freq > 0.0) || !std::isfinite(h) ||
        !std::isfinite(freq))
        return HELM27_EINVAL;
    if (n <= 0 || n > kNaMaxPoints) {
        std::fprintf(stderr, "helm27_select_index_noalloc: %lld points; its scratch holds at most %lld\n",
                     static_cast<long long>(n), static_cast<long long>(kNaMaxPoints));
        return HELM27_EINVAL;
    }
    int prev = 0;
    H27_CHECK_HIP(hipGetDevice(&prev));
    if (prev != ctx->device) H27_CHECK_HIP(hipSetDevice(ctx->device));
    auto done = [&](int st) {
        if (prev != ctx->device) (void)hipSetDevice(prev);
        return st;
    };
    if (!device_pointer_on(vel, ctx->device) || !device_pointer_on(idx, ctx->device)) return done(HELM27_EINVAL);
    NaRecord* rec = nullptr;
    int st = scratch_address(ctx->device, &rec);
    if (st) return done(st);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nblocks = static_cast<int>((n + kNaPerBlock - 1) / kNaPerBlock);
    const double fh = freq * h;
    hipLaunchKernelGGL(select_index_blocks_kernel, dim3(nblocks), dim3(kBlock), 0, s, vel, idx, n, fh, t->g_min,
                       t->dg, t->n_g, t->spacing, rec);
    if (hipGetLastError() != hipSuccess) return done(HELM27_EDEVICE);
    hipLaunchKernelGGL(reduce_records_kernel, dim3(1), dim3(kBlock), 0, s, rec, nblocks, rec + kNaBlocks);
    if (hipGetLastError() != hipSuccess) return done(HELM27_EDEVICE);
    if (!stats) return done(HELM27_OK);
    NaRecord r{};
    if (hipMemcpyAsync(&r, rec + kNaBlocks, sizeof(r), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return done(HELM27_EDEVICE);
    float cmin = __builtin_inff(), cmax = 0.0f;
    const unsigned lo = static_cast<unsigned>(r.minbits), hi = static_cast<unsigned>(r.maxbits);
    std::memcpy(&cmin, &lo, sizeof(float));
    std::memcpy(&cmax, &hi, sizeof(float));
    stats->n_clamped = static_cast<int64_t>(r.ncl);
    stats->n_invalid = static_cast<int64_t>(r.nbad);
    stats->g_min_model = static_cast<double>(cmin) / fh;   // G = c/(f h) on either table axis
    stats->g_max_model = static_cast<double>(cmax) / fh;
    return done(r.nbad ? HELM27_EINVAL : HELM27_OK);
}
