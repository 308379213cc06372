// 27-point stencil over the plain box (x and y unstretched; z may be
// stretched).  Same operator and in-plane decomposition as the tiled kernel
// in kernels_stencil.hip (centre / 4-face sum / 4-diagonal sum per plane,
// 9-term combination per output row), organised for latency hiding on CDNA:
//
//   * one wavefront per work item (62 output columns x RY rows x a z chunk x
//     one right-hand side); no block barriers inside the z march;
//   * x neighbours by cross-lane DPP shifts of the wave's 64 loaded columns
//     (lanes 0 and 63 are halo lanes and produce no output), y neighbours by
//     loading RY + 2 rows per plane, z neighbours from registers;
//   * every global load is unconditional (clamped address, then zeroed if
//     outside the grid) and every store is unconditional (lanes without an
//     output write to a 64-entry sink buffer), so the memory counters stay
//     exact and the next plane's loads and the next output plane's table
//     index / velocity are in flight during the current plane's arithmetic;
//   * the slice of the weight table that the grid uses is staged in LDS once
//     per block, so the per-row table lookup is an LDS read.
#include "stencil.h"

namespace h27 {

template <typename R>
struct TabEntry {
    R s[4];
    R m[4];
};

// lane i <- lane i + 1 and lane i <- lane i - 1 across the whole wavefront
__device__ __forceinline__ float wshl(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float wshr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double wshl(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double wshr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <typename R>
__device__ __forceinline__ Cx<R> xpair(Cx<R> v) {
    return Cx<R>{wshl(v.re) + wshr(v.re), wshl(v.im) + wshr(v.im)};
}

template <typename R, int MODE, bool SHIFTED, int RY>
__global__ __launch_bounds__(kBlock) void plain27_kernel(PlainArgs<R> a) {
    using V = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TabEntry<R>* tab = reinterpret_cast<TabEntry<R>*>(smem_raw);
    const GridData<R>& g = a.g;
    for (int t = threadIdx.x; t < a.n_tab; t += kBlock) {
        const EntryCoef<R> E = g.entry[a.tab_lo + t];
        TabEntry<R> e;
        e.s[0] = E.s0; e.s[1] = E.s1; e.s[2] = E.s2; e.s[3] = E.s3;
        e.m[0] = E.m0; e.m[1] = E.m1; e.m[2] = E.m2; e.m[3] = E.m3;
        tab[t] = e;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = blockIdx.x * (kBlock / 64) + wave;
    if (item >= a.n_items) return;
    int t = item;
    const int tx = t % a.ntx;
    t /= a.ntx;
    const int ty = t % a.nty;
    t /= a.nty;
    const int zc = t % a.nzc;
    const int rhs = t / a.nzc;

    const int gx = a.px0 + tx * kWaveCols - 1 + lane;
    const bool outx = lane >= 1 && lane <= kWaveCols && gx < a.px0 + a.pw;
    const bool inx = gx >= 0 && gx < g.nx;
    const int gxc = min(max(gx, 0), g.nx - 1);
    const int y0 = a.py0 + ty * RY;
    const int z0 = zc * a.zchunk;
    const int z1 = min(z0 + a.zchunk, g.nz);
    const int yend = a.py0 + a.ph;

    int off[RY + 2];
    bool okk[RY + 2];
#pragma unroll
    for (int k = 0; k < RY + 2; ++k) {
        const int yy = y0 - 1 + k;
        okk[k] = inx && yy >= 0 && yy < g.ny;
        off[k] = min(max(yy, 0), g.ny - 1) * g.nx + gxc;
    }
    const V* u = a.u + static_cast<int64_t>(rhs) * g.N;
    V* const yrhs = a.y + static_cast<int64_t>(rhs) * g.N;
    V* const sink = a.sink + lane;
    const V* bvec = (MODE == MODE_APPLY) ? nullptr : a.b + static_cast<int64_t>(rhs) * g.N;

    auto load_plane = [&](int q, Cx<R>(&dst)[RY + 2]) {
        const bool okq = q >= 0 && q < g.nz;
        const int qc = min(max(q, 0), g.nz - 1);
        const V* p = u + static_cast<int64_t>(qc) * g.plane;
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) {
            const V v = p[off[k]];
            const bool ok = okq && okk[k];
            dst[k] = Cx<R>{ok ? v.x : R(0), ok ? v.y : R(0)};
        }
    };
    auto load_meta = [&](int q, int (&idx)[RY], float (&cv)[RY]) {
        const int64_t pb = static_cast<int64_t>(q) * g.plane;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int64_t i = pb + off[r + 1];
            idx[r] = g.fixed ? 0 : static_cast<int>(g.idx[i]);
            cv[r] = g.c[i];
        }
    };

    Cx<R> U[RY + 2];
    load_plane(z0 - 1, U);
    int idxN[RY];
    float cN[RY];
    load_meta(z0, idxN, cN);
    Cx<R> Ac[RY], Af[RY], Ae[RY], Bc[RY], Bf[RY], Be[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) Ac[r] = Af[r] = Ae[r] = Bc[r] = Bf[r] = Be[r] = zero<R>();

    for (int q = z0 - 1; q <= z1; ++q) {
        // in-plane decomposition of plane q
        Cx<R> m[RY + 2], sx[RY + 2];
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) {
            m[k] = U[k];
            sx[k] = xpair(U[k]);
        }
        Cx<R> Cc[RY], Cf[RY], Ce[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            Cc[r] = m[r + 1];
            Cf[r] = sx[r + 1] + m[r] + m[r + 2];
            Ce[r] = sx[r] + sx[r + 2];
        }
        if (q + 1 <= z1) load_plane(q + 1, U);
        if (q >= z0 + 1) {
            const int zo = q - 1;
            int idxM[RY];
            float cM[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                idxM[r] = idxN[r];
                cM[r] = cN[r];
            }
            if (q < z1) load_meta(q, idxN, cN);
            const AxisNode<R> Z = g.az[zo];
            const R sig = g.inv_h2;
            const int64_t pb = static_cast<int64_t>(zo) * g.plane;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const TabEntry<R> E = tab[idxM[r] - a.tab_lo];
                const R cvr = static_cast<R>(cM[r]);
                const R kap = g.omega2 / (cvr * cvr);
                Cx<R> acc = zero<R>(), diag = zero<R>();
                if (Z.plain) {
                    const Cx<R> Fc = Bf[r] + Ac[r] + Cc[r];
                    const Cx<R> Ec = Be[r] + Af[r] + Cf[r];
                    const Cx<R> Co = Ae[r] + Ce[r];
                    const R A0 = sig * E.s[0] + kap * E.m[0], A1 = sig * E.s[1] + kap * E.m[1];
                    const R A2 = sig * E.s[2] + kap * E.m[2], A3 = sig * E.s[3] + kap * E.m[3];
                    if (SHIFTED) {
                        const R kr = kap * (g.shift_re - R(1)), ks = kap * g.shift_im;
                        const Cx<R> K0{A0 + kr * E.m[0], ks * E.m[0]}, K1{A1 + kr * E.m[1], ks * E.m[1]};
                        const Cx<R> K2{A2 + kr * E.m[2], ks * E.m[2]}, K3{A3 + kr * E.m[3], ks * E.m[3]};
                        cmac(acc, K0, Bc[r]);
                        cmac(acc, K1, Fc);
                        cmac(acc, K2, Ec);
                        cmac(acc, K3, Co);
                        diag = K0;
                    } else {
                        rmac(acc, A0, Bc[r]);
                        rmac(acc, A1, Fc);
                        rmac(acc, A2, Ec);
                        rmac(acc, A3, Co);
                        diag = Cx<R>{A0, R(0)};
                    }
                } else {
                    const R b2 = E.s[2] + R(2) * E.s[3];   // beta2 = s2 + 2 s3
                    const Cx<R> tm{Z.tm_re, Z.tm_im}, tp{Z.tp_re, Z.tp_im};
                    const Cx<R> t0 = -(tm + tp);
                    const Cx<R> xz{Z.xi_re, Z.xi_im};
                    const Cx<R> um{Z.um_re, Z.um_im}, up{Z.up_re, Z.up_im};
                    const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
                    const Cx<R> kum = kc * um, kup = kc * up, kxz = kc * xz;
                    const Cx<R> Kcm = (sig * E.s[1]) * tm + (R(2) * E.m[1]) * kum;
                    const Cx<R> Kfm = (sig * E.s[2]) * tm + (R(2) * E.m[2]) * kum;
                    const Cx<R> Kem = (sig * E.s[3]) * tm + (R(2) * E.m[3]) * kum;
                    const Cx<R> Kcp = (sig * E.s[1]) * tp + (R(2) * E.m[1]) * kup;
                    const Cx<R> Kfp = (sig * E.s[2]) * tp + (R(2) * E.m[2]) * kup;
                    const Cx<R> Kep = (sig * E.s[3]) * tp + (R(2) * E.m[3]) * kup;
                    const Cx<R> Kc0 = (sig * E.s[1]) * t0 + (sig * (R(4) * b2 - R(4))) * xz + E.m[0] * kxz;
                    const Cx<R> Kf0 = (sig * E.s[2]) * t0 + (sig * (R(1) - R(2) * b2)) * xz + E.m[1] * kxz;
                    const Cx<R> Ke0 = (sig * E.s[3]) * t0 + (sig * b2) * xz + E.m[2] * kxz;
                    cmac(acc, Kcm, Ac[r]);
                    cmac(acc, Kfm, Af[r]);
                    cmac(acc, Kem, Ae[r]);
                    cmac(acc, Kc0, Bc[r]);
                    cmac(acc, Kf0, Bf[r]);
                    cmac(acc, Ke0, Be[r]);
                    cmac(acc, Kcp, Cc[r]);
                    cmac(acc, Kfp, Cf[r]);
                    cmac(acc, Kep, Ce[r]);
                    diag = Kc0;
                }
                const bool valid = outx && (y0 + r < yend);
                const int64_t i = pb + off[r + 1];
                Cx<R> outv = acc;
                if (MODE != MODE_APPLY) {
                    const V bb = bvec[i];
                    const Cx<R> rr{bb.x - acc.re, bb.y - acc.im};
                    if (MODE == MODE_RESID) {
                        outv = rr;
                    } else {
                        outv = Bc[r] + a.omega_j * (rr * cinv(diag));
                    }
                }
                V* dst = valid ? yrhs + i : sink;
                V ov;
                ov.x = outv.re;
                ov.y = outv.im;
                *dst = ov;
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            Ac[r] = Bc[r]; Af[r] = Bf[r]; Ae[r] = Be[r];
            Bc[r] = Cc[r]; Bf[r] = Cf[r]; Be[r] = Ce[r];
        }
    }
}

template <typename R, int MODE, bool SHIFTED, int RY>
static int launch_plain_ry(const PlainArgs<R>& a, hipStream_t s) {
    const int blocks = (a.n_items + (kBlock / 64) - 1) / (kBlock / 64);
    const size_t lds = static_cast<size_t>(a.n_tab) * sizeof(TabEntry<R>);
    hipLaunchKernelGGL((plain27_kernel<R, MODE, SHIFTED, RY>), dim3(blocks), dim3(kBlock), lds, s, a);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

template <typename R, int MODE, bool SHIFTED>
static int launch_plain_mode(const PlainArgs<R>& a, int ry, hipStream_t s) {
    switch (ry) {
        case 1: return launch_plain_ry<R, MODE, SHIFTED, 1>(a, s);
        case 2: return launch_plain_ry<R, MODE, SHIFTED, 2>(a, s);
        case 3: return launch_plain_ry<R, MODE, SHIFTED, 3>(a, s);
        case 4: return launch_plain_ry<R, MODE, SHIFTED, 4>(a, s);
        default: return HELM27_EINVAL;
    }
}

template <typename R>
int launch_plain(const PlainArgs<R>& a, int mode, bool shifted, int ry, hipStream_t s) {
    if (a.n_items <= 0) return HELM27_OK;
    switch (mode) {
        case MODE_APPLY:
            return shifted ? launch_plain_mode<R, MODE_APPLY, true>(a, ry, s)
                           : launch_plain_mode<R, MODE_APPLY, false>(a, ry, s);
        case MODE_RESID:
            return shifted ? launch_plain_mode<R, MODE_RESID, true>(a, ry, s)
                           : launch_plain_mode<R, MODE_RESID, false>(a, ry, s);
        case MODE_JACOBI:
            return shifted ? launch_plain_mode<R, MODE_JACOBI, true>(a, ry, s)
                           : launch_plain_mode<R, MODE_JACOBI, false>(a, ry, s);
        default:
            return HELM27_EINVAL;
    }
}
template int launch_plain<float>(const PlainArgs<float>&, int, bool, int, hipStream_t);
template int launch_plain<double>(const PlainArgs<double>&, int, bool, int, hipStream_t);

}  // namespace h27
