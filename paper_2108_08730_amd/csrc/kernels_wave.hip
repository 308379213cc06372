// Wavefront-per-tile 27-point stencil (apply, residual, damped Jacobi).
//
// Operator (paper Sec. 2.1 with per-row weights, Sec. 3.1): for an output row
// with table entry E and kappa = k^2 (a + i b) ((a, b) = (1, 0) for the
// physical operator),
//   A u = (1/h^2) [ sum_a T_a + beta2 sum_{a<b} T_a T_b + beta3 T_x T_y T_z ] u
//       + kappa   [ m0 XXX + 2 m1 sum UXX + 4 m2 sum UUX + 8 m3 UUU ] u
// with T, U, X the (stretched) 1D second difference, neighbour half-sum and
// node stretch; an axis absent from a product contributes X.
//
// One wavefront per work item: 62 output columns along its lane axis (lanes
// 0 and 63 are halo), R rows along the other in-plane axis, a chunk of z
// planes marched in registers, one right-hand side.
//   * In-plane neighbours along the lane axis come from cross-lane DPP shifts
//     of the values the wave loaded, along the row axis from the R + 2 rows it
//     loads per plane, along z from the previous planes kept in registers.
//   * Every global load is unconditional (clamped address, zeroed outside the
//     grid) and every store is unconditional (masked lanes write a 64-entry
//     sink), so the memory counters stay exact: the next plane's loads and the
//     next output plane's table index / velocity are in flight during the
//     current plane's arithmetic.
//   * The slice of the weight table the grid uses is staged in LDS per block.
// Two kinds of work items share a launch:
//   * box tiles (x and y unstretched, lanes along x): per plane the centre c,
//     4-face sum f and 4-diagonal sum e; the output is a 9-term combination
//     with real coefficients, complex in z-PML planes (uniform per plane);
//   * PML-frame tiles (lanes along x in the y-strips, along y in the
//     x-strips): the separable contractions a = XX u, b = (TX + XT) u,
//     c = TT u, d = (UX + XU) u, e = UU u with the complex 1D factors of the
//     lane node and of the row node, then the same z combination.
#include "stencil.h"

namespace h27 {

template <typename R>
struct TabEntry {
    R s[4];
    R m[4];
};

// lane i <- lane i + 1 (wshl) and lane i <- lane i - 1 (wshr), whole wavefront
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
// the same within each row of 16 lanes
__device__ __forceinline__ float rshl(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, true));
}
__device__ __forceinline__ float rshr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
}
__device__ __forceinline__ double rshl(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x101, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x101, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double rshr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x111, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x111, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <typename R>
__device__ __forceinline__ Cx<R> nxt(Cx<R> v) { return Cx<R>{wshl(v.re), wshl(v.im)}; }   // lane + 1
template <typename R>
__device__ __forceinline__ Cx<R> prv(Cx<R> v) { return Cx<R>{wshr(v.re), wshr(v.im)}; }   // lane - 1
// neighbours along x for a lane-group width of 64 (whole wave) or 16 (DPP rows)
template <int LW, typename R>
__device__ __forceinline__ Cx<R> nxt_g(Cx<R> v) {
    if (LW == 64) return nxt(v);
    return Cx<R>{rshl(v.re), rshl(v.im)};
}
template <int LW, typename R>
__device__ __forceinline__ Cx<R> prv_g(Cx<R> v) {
    if (LW == 64) return prv(v);
    return Cx<R>{rshr(v.re), rshr(v.im)};
}

template <typename R>
__device__ __forceinline__ Cx<R> cz(R re, R im) { return Cx<R>{re, im}; }

template <typename R, int MODE>
__device__ __forceinline__ void wave_store(const WaveArgs<R>& a, typename V2<R>::T* yrhs,
                                           const typename V2<R>::T* brhs, typename V2<R>::T* sink, bool valid,
                                           int64_t i, Cx<R> acc, Cx<R> diag, Cx<R> xcen) {
    using V = typename V2<R>::T;
    Cx<R> outv = acc;
    if (MODE != MODE_APPLY) {
        const V bb = brhs[i];
        const Cx<R> rr{bb.x - acc.re, bb.y - acc.im};
        if (MODE == MODE_RESID) outv = rr;
        else outv = xcen + a.omega_j * (rr * cinv(diag));
    }
    V* dst = valid ? yrhs + i : sink;
    V ov;
    ov.x = outv.re;
    ov.y = outv.im;
    *dst = ov;
}

// ---------------------------------------------------------------------------
// unstretched-box tile
template <typename R, int MODE, bool SHIFTED, int RY>
__device__ __forceinline__ void box_item(const WaveArgs<R>& a, const TabEntry<R>* tab, int tile, int zc, int rhs,
                                         int lane) {
    using V = typename V2<R>::T;
    const GridData<R>& g = a.g;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
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
    const V* brhs = (MODE == MODE_APPLY) ? nullptr : a.b + static_cast<int64_t>(rhs) * g.N;
    V* const sink = a.sink + lane;

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
        Cx<R> sx[RY + 2];
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) sx[k] = nxt(U[k]) + prv(U[k]);
        Cx<R> Cc[RY], Cf[RY], Ce[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            Cc[r] = U[r + 1];
            Cf[r] = sx[r + 1] + U[r] + U[r + 2];
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
                TabEntry<R> E;
                if (g.rowcoef) {
                    const EntryCoef<R> F = g.rowcoef[pb + off[r + 1]];
                    E.s[0] = F.s0; E.s[1] = F.s1; E.s[2] = F.s2; E.s[3] = F.s3;
                    E.m[0] = F.m0; E.m[1] = F.m1; E.m[2] = F.m2; E.m[3] = F.m3;
                } else {
                    E = tab[idxM[r] - a.tab_lo];
                }
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
                wave_store<R, MODE>(a, yrhs, brhs, sink, valid, pb + off[r + 1], acc, diag, Bc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            Ac[r] = Bc[r]; Af[r] = Bf[r]; Ae[r] = Be[r];
            Bc[r] = Cc[r]; Bf[r] = Cf[r]; Be[r] = Ce[r];
        }
    }
}

// ---------------------------------------------------------------------------
// PML-frame tile: lanes along x (lx) or along y (!lx)
template <typename R>
struct Factors {
    Cx<R> tm, tp, t0, xi, um, up;
};
template <typename R>
__device__ __forceinline__ Factors<R> factors(const AxisNode<R>& n) {
    Factors<R> f;
    f.tm = Cx<R>{n.tm_re, n.tm_im};
    f.tp = Cx<R>{n.tp_re, n.tp_im};
    f.t0 = -(f.tm + f.tp);
    f.xi = Cx<R>{n.xi_re, n.xi_im};
    f.um = Cx<R>{n.um_re, n.um_im};
    f.up = Cx<R>{n.up_re, n.up_im};
    return f;
}

template <typename R, int MODE, bool SHIFTED, int RQ, int LW>
__device__ __forceinline__ void frame_item(const WaveArgs<R>& a, const TabEntry<R>* tab, int fr, int ft, int zc,
                                           int rhs, int lane) {
    using V = typename V2<R>::T;
    const GridData<R>& g = a.g;
    // lanes along x in groups of LW (LW - 2 output columns each, halo at both
    // ends), 64 / LW groups stacked along y, RQ rows per lane
    constexpr int NG = 64 / LW;
    const int lx = lane % LW, ly = lane / LW;
    const int tl = ft % a.fnl[fr], tq = ft / a.fnl[fr];
    const int x_org = a.fx0[fr], x_ext = a.fw[fr];
    const int y_org = a.fy0[fr], y_ext = a.fh[fr];
    const int lc = x_org + tl * (LW - 2) - 1 + lx;
    const bool outl = lx >= 1 && lx <= LW - 2 && lc < x_org + x_ext;
    const bool inl = lc >= 0 && lc < g.nx;
    const int lcc = min(max(lc, 0), g.nx - 1);
    const int q0 = y_org + (tq * NG + ly) * RQ;
    const int z0 = zc * a.zchunk;
    const int z1 = min(z0 + a.zchunk, g.nz);
    const Factors<R> FL = factors<R>(g.ax[lcc]);
    Factors<R> FQ[RQ];
    Cx<R> xLQ[RQ];
    int off[RQ + 2];
    bool okk[RQ + 2];
#pragma unroll
    for (int k = 0; k < RQ + 2; ++k) {
        const int qq = q0 - 1 + k;
        okk[k] = inl && qq >= 0 && qq < g.ny;
        off[k] = min(max(qq, 0), g.ny - 1) * g.nx + lcc;
    }
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        FQ[r] = factors<R>(g.ay[min(q0 + r, g.ny - 1)]);
        xLQ[r] = FL.xi * FQ[r].xi;
    }
    const V* u = a.u + static_cast<int64_t>(rhs) * g.N;
    V* const yrhs = a.y + static_cast<int64_t>(rhs) * g.N;
    const V* brhs = (MODE == MODE_APPLY) ? nullptr : a.b + static_cast<int64_t>(rhs) * g.N;
    V* const sink = a.sink + lane;

    auto load_plane = [&](int q, Cx<R>(&dst)[RQ + 2]) {
        const bool okq = q >= 0 && q < g.nz;
        const int qc = min(max(q, 0), g.nz - 1);
        const V* p = u + static_cast<int64_t>(qc) * g.plane;
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) {
            const V v = p[off[k]];
            const bool ok = okq && okk[k];
            dst[k] = Cx<R>{ok ? v.x : R(0), ok ? v.y : R(0)};
        }
    };
    auto load_meta = [&](int q, int (&idx)[RQ], float (&cv)[RQ]) {
        const int64_t pb = static_cast<int64_t>(q) * g.plane;
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            const int64_t i = pb + off[r + 1];
            idx[r] = g.fixed ? 0 : static_cast<int>(g.idx[i]);
            cv[r] = g.c[i];
        }
    };

    Cx<R> U[RQ + 2];
    load_plane(z0 - 1, U);
    int idxN[RQ];
    float cN[RQ];
    load_meta(z0, idxN, cN);
    // contractions of planes q-2 (A) and q-1 (B), and the centre value of B
    Cx<R> aA[RQ], bA[RQ], cA[RQ], dA[RQ], eA[RQ], aB[RQ], bB[RQ], cB[RQ], dB[RQ], eB[RQ], uB[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r)
        aA[r] = bA[r] = cA[r] = dA[r] = eA[r] = aB[r] = bB[r] = cB[r] = dB[r] = eB[r] = uB[r] = zero<R>();

    for (int q = z0 - 1; q <= z1; ++q) {
        Cx<R> RT[RQ + 2], RU[RQ + 2];
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) {
            const Cx<R> vm = prv_g<LW>(U[k]), vp = nxt_g<LW>(U[k]);
            RT[k] = FL.tm * vm + FL.t0 * U[k] + FL.tp * vp;
            RU[k] = FL.um * vm + FL.up * vp;
        }
        Cx<R> aC[RQ], bC[RQ], cC[RQ], dC[RQ], eC[RQ], uC[RQ];
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            const Factors<R>& Q = FQ[r];
            uC[r] = U[r + 1];
            aC[r] = xLQ[r] * U[r + 1];
            bC[r] = Q.xi * RT[r + 1] + FL.xi * (Q.tm * U[r] + Q.t0 * U[r + 1] + Q.tp * U[r + 2]);
            cC[r] = Q.tm * RT[r] + Q.t0 * RT[r + 1] + Q.tp * RT[r + 2];
            dC[r] = Q.xi * RU[r + 1] + FL.xi * (Q.um * U[r] + Q.up * U[r + 2]);
            eC[r] = Q.um * RU[r] + Q.up * RU[r + 2];
        }
        if (q + 1 <= z1) load_plane(q + 1, U);
        if (q >= z0 + 1) {
            const int zo = q - 1;
            int idxM[RQ];
            float cM[RQ];
#pragma unroll
            for (int r = 0; r < RQ; ++r) {
                idxM[r] = idxN[r];
                cM[r] = cN[r];
            }
            if (q < z1) load_meta(q, idxN, cN);
            const Factors<R> FZ = factors<R>(g.az[zo]);
            const R sig = g.inv_h2;
            const int64_t pb = static_cast<int64_t>(zo) * g.plane;
#pragma unroll
            for (int r = 0; r < RQ; ++r) {
                R b2, b3, m0, m1, m2, m3;
                if (g.rowcoef) {
                    const EntryCoef<R> E = g.rowcoef[pb + off[r + 1]];
                    b2 = E.beta2; b3 = E.beta3; m0 = E.m0; m1 = E.m1; m2 = E.m2; m3 = E.m3;
                } else {
                    const TabEntry<R> E = tab[idxM[r] - a.tab_lo];
                    b3 = E.s[3];
                    b2 = E.s[2] + R(2) * E.s[3];
                    m0 = E.m[0]; m1 = E.m[1]; m2 = E.m[2]; m3 = E.m[3];
                }
                const R cvr = static_cast<R>(cM[r]);
                const R kap = g.omega2 / (cvr * cvr);
                const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
                Cx<R> PTA = aA[r], PTB = aB[r], PTC = aC[r];
                rmac(PTA, b2, bA[r]); rmac(PTA, b3, cA[r]);
                rmac(PTB, b2, bB[r]); rmac(PTB, b3, cB[r]);
                rmac(PTC, b2, bC[r]); rmac(PTC, b3, cC[r]);
                Cx<R> PUA = zero<R>(), PUC = zero<R>();
                rmac(PUA, R(2) * m1, aA[r]); rmac(PUA, R(4) * m2, dA[r]); rmac(PUA, R(8) * m3, eA[r]);
                rmac(PUC, R(2) * m1, aC[r]); rmac(PUC, R(4) * m2, dC[r]); rmac(PUC, R(8) * m3, eC[r]);
                Cx<R> PXs = bB[r];
                rmac(PXs, b2, cB[r]);
                Cx<R> PXm = zero<R>();
                rmac(PXm, m0, aB[r]); rmac(PXm, R(2) * m1, dB[r]); rmac(PXm, R(4) * m2, eB[r]);
                Cx<R> stiff = FZ.tm * PTA;
                cmac(stiff, FZ.t0, PTB);
                cmac(stiff, FZ.tp, PTC);
                cmac(stiff, FZ.xi, PXs);
                Cx<R> mass = FZ.um * PUA;
                cmac(mass, FZ.up, PUC);
                cmac(mass, FZ.xi, PXm);
                Cx<R> acc = sig * stiff;
                cmac(acc, kc, mass);
                Cx<R> diag = zero<R>();
                if (MODE == MODE_JACOBI) {
                    const Factors<R>& Q = FQ[r];
                    const Cx<R> ac = xLQ[r];
                    const Cx<R> bc = FL.t0 * Q.xi + FL.xi * Q.t0;
                    const Cx<R> cc = FL.t0 * Q.t0;
                    Cx<R> pc = ac;
                    rmac(pc, b2, bc);
                    rmac(pc, b3, cc);
                    Cx<R> pxs = bc;
                    rmac(pxs, b2, cc);
                    diag = sig * (FZ.t0 * pc + FZ.xi * pxs) + (m0 * kc) * (FZ.xi * ac);
                }
                const bool valid = outl && (q0 + r < y_org + y_ext);
                wave_store<R, MODE>(a, yrhs, brhs, sink, valid, pb + off[r + 1], acc, diag, uB[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            aA[r] = aB[r]; bA[r] = bB[r]; cA[r] = cB[r]; dA[r] = dB[r]; eA[r] = eB[r];
            aB[r] = aC[r]; bB[r] = bC[r]; cB[r] = cC[r]; dB[r] = dC[r]; eB[r] = eC[r];
            uB[r] = uC[r];
        }
    }
}

template <typename R, int MODE, bool SHIFTED, int RY, int RQ, int WHICH>
__global__ __launch_bounds__(kBlock) void wave27_kernel(WaveArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TabEntry<R>* tab = reinterpret_cast<TabEntry<R>*>(smem_raw);
    const GridData<R>& g = a.g;
    if (!g.rowcoef) {
        for (int t = threadIdx.x; t < a.n_tab; t += kBlock) {
            const EntryCoef<R> E = g.entry[a.tab_lo + t];
            TabEntry<R> e;
            e.s[0] = E.s0; e.s[1] = E.s1; e.s[2] = E.s2; e.s[3] = E.s3;
            e.m[0] = E.m0; e.m[1] = E.m1; e.m[2] = E.m2; e.m[3] = E.m3;
            tab[t] = e;
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = blockIdx.x * (kBlock / 64) + wave;
    if (item >= a.n_items) return;
    const int ntile = (WHICH == WAVE_PLAIN ? 0 : a.n_frame) + (WHICH == WAVE_FRAME ? 0 : a.n_plain);
    const int tile = item % ntile;
    const int t = item / ntile;
    const int zc = t % a.nzc;
    const int rhs = t / a.nzc;
    if (WHICH != WAVE_PLAIN && tile < a.n_frame) {
        int k = 0;
        while (k < 3 && tile >= a.fstart[k + 1]) ++k;
        if (a.flx[k])
            frame_item<R, MODE, SHIFTED, RQ, 64>(a, tab, k, tile - a.fstart[k], zc, rhs, lane);
        else
            frame_item<R, MODE, SHIFTED, RQ, 16>(a, tab, k, tile - a.fstart[k], zc, rhs, lane);
    } else if (WHICH != WAVE_FRAME) {
        box_item<R, MODE, SHIFTED, RY>(a, tab, tile - (WHICH == WAVE_PLAIN ? 0 : a.n_frame), zc, rhs, lane);
    }
}

template <typename R> struct FrameRows;
template <> struct FrameRows<float> { static constexpr int value = 1; };
template <> struct FrameRows<double> { static constexpr int value = 1; };

template <typename R, int MODE, bool SHIFTED, int RY>
static int launch_wave_ry(const WaveArgs<R>& a, hipStream_t s) {
    constexpr int RQ = FrameRows<R>::value;
    const int blocks = (a.n_items + (kBlock / 64) - 1) / (kBlock / 64);
    const size_t lds = a.g.rowcoef ? 16 : static_cast<size_t>(a.n_tab) * sizeof(TabEntry<R>);
    if (a.n_frame > 0 && a.n_plain > 0)
        hipLaunchKernelGGL((wave27_kernel<R, MODE, SHIFTED, RY, RQ, WAVE_BOTH>), dim3(blocks), dim3(kBlock), lds, s, a);
    else if (a.n_plain > 0)
        hipLaunchKernelGGL((wave27_kernel<R, MODE, SHIFTED, RY, RQ, WAVE_PLAIN>), dim3(blocks), dim3(kBlock), lds, s, a);
    else
        hipLaunchKernelGGL((wave27_kernel<R, MODE, SHIFTED, RY, RQ, WAVE_FRAME>), dim3(blocks), dim3(kBlock), lds, s, a);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

template <typename R, int MODE, bool SHIFTED>
static int launch_wave_mode(const WaveArgs<R>& a, int ry, hipStream_t s) {
    switch (ry) {
        case 1: return launch_wave_ry<R, MODE, SHIFTED, 1>(a, s);
        case 2: return launch_wave_ry<R, MODE, SHIFTED, 2>(a, s);
        case 3: return launch_wave_ry<R, MODE, SHIFTED, 3>(a, s);
        case 4: return launch_wave_ry<R, MODE, SHIFTED, 4>(a, s);
        default: return HELM27_EINVAL;
    }
}

template <typename R>
int launch_wave(const WaveArgs<R>& a, int mode, bool shifted, int ry, int rq, hipStream_t s) {
    (void)rq;
    if (a.n_items <= 0) return HELM27_OK;
    switch (mode) {
        case MODE_APPLY:
            return shifted ? launch_wave_mode<R, MODE_APPLY, true>(a, ry, s)
                           : launch_wave_mode<R, MODE_APPLY, false>(a, ry, s);
        case MODE_RESID:
            return shifted ? launch_wave_mode<R, MODE_RESID, true>(a, ry, s)
                           : launch_wave_mode<R, MODE_RESID, false>(a, ry, s);
        case MODE_JACOBI:
            return shifted ? launch_wave_mode<R, MODE_JACOBI, true>(a, ry, s)
                           : launch_wave_mode<R, MODE_JACOBI, false>(a, ry, s);
        default:
            return HELM27_EINVAL;
    }
}
template int launch_wave<float>(const WaveArgs<float>&, int, bool, int, int, hipStream_t);
template int launch_wave<double>(const WaveArgs<double>&, int, bool, int, int, hipStream_t);

template <typename R>
int frame_rows() { return FrameRows<R>::value; }
template int frame_rows<float>();
template int frame_rows<double>();

}  // namespace h27
