#pragma once
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
//   * All control flow is wave-uniform (scalar registers): the work item, the
//     z loop, the plane kind, the row count and the grid-edge case.
//   * In-plane neighbours along the lane axis come from cross-lane DPP shifts
//     of the values the wave loaded, along the row axis from the R + 2 rows it
//     loads per plane, along z from the previous planes kept in registers.
//   * Software pipeline: the loads of plane q + 2 and the per-point data of
//     output plane q are issued before plane q is combined; loads go to
//     clamped (always valid) addresses and the zero outside the grid is
//     applied when the plane is used.  The z loop is unrolled three times so
//     the three load buffers, plane slots and per-point slots rotate by
//     renaming, not copying.
//   * The slice of the weight table the grid uses is staged in LDS per block
//     (stiffness weights pre-scaled by 1/h^2).
//   * Blocks are renumbered so that each XCD (blocks dispatched round-robin
//     over the 8 XCDs) runs a contiguous range of work items, and rows shared
//     by neighbouring tiles are re-read from its own L2.
// Two kinds of work items share a launch:
//   * box tiles (x and y unstretched, lanes along x): per plane the centre c,
//     4-face sum f and 4-diagonal sum e; the output is a 9-term combination
//     with real coefficients, complex in z-PML planes (uniform per plane);
//   * PML-frame tiles (lanes along x in groups of 64 or 16): the separable
//     contractions a = XX u, b = (TX + XT) u, c = TT u, d = (UX + XU) u,
//     e = UU u with the complex 1D factors of the lane node and of the row
//     node, then the same z combination.
#include "stencil.h"

namespace h27 {

// LDS copy of one table entry: s = stiffness class weights times 1/h^2,
// m = mass class weights, b2 / b3 = unscaled beta2 / beta3 (frame formula).
template <typename R>
struct alignas(16) TabEntry {
    R s[4];
    R m[4];
    R b2, b3, pad0, pad1;
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
// neighbours along the lane axis for a lane-group width of 64 (whole wave) or 16 (DPP rows)
template <int LW, typename R>
__device__ __forceinline__ Cx<R> nxt_g(Cx<R> v) {
    if (LW == 64) return Cx<R>{wshl(v.re), wshl(v.im)};
    return Cx<R>{rshl(v.re), rshl(v.im)};
}
template <int LW, typename R>
__device__ __forceinline__ Cx<R> prv_g(Cx<R> v) {
    if (LW == 64) return Cx<R>{wshr(v.re), wshr(v.im)};
    return Cx<R>{rshr(v.re), rshr(v.im)};
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// reciprocal: v_rcp_f32 (1 ulp) in the FP32 kernels, a correctly rounded
// division in the FP64 kernels
__device__ __forceinline__ float rcp_of(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_of(double x) { return 1.0 / x; }

template <typename R>
__device__ __forceinline__ Cx<R> inv_of(Cx<R> a) {
    const R d = rcp_of(a.re * a.re + a.im * a.im);
    return Cx<R>{a.re * d, -a.im * d};
}

// the value a mode stores for the operator row acc = (A u)_i
template <typename R, int MODE>
__device__ __forceinline__ Cx<R> finish(R omega_j, Cx<R> acc, Cx<R> diag, Cx<R> xcen,
                                        typename V2<R>::T bb) {
    if (MODE == MODE_APPLY) return acc;
    if (MODE == MODE_JACOBI0) return omega_j * (Cx<R>{bb.x, bb.y} * inv_of(diag));
    const Cx<R> rr{bb.x - acc.re, bb.y - acc.im};
    if (MODE == MODE_RESID) return rr;
    return xcen + omega_j * (rr * inv_of(diag));
}

// ---------------------------------------------------------------------------
// Buffer loads and stores.  Every vector access goes through a buffer resource
// with the byte size of its array, so the hardware range check does the grid
// boundary: a lane offset of kOff (or a plane outside the grid, whose
// resource has size 0) reads 0 and drops the store; no lane masks, no
// address arithmetic in the vector unit.
using Rsrc = __amdgpu_buffer_rsrc_t;
using u32x2 = unsigned int __attribute__((ext_vector_type(2)));
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;          // untyped 32-bit data, range checked
constexpr unsigned kOff = 0x80000000u;          // beyond every buffer (sizes < 2^31 bytes)

__device__ __forceinline__ Rsrc rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), kRsrcWord3);
}
__device__ __forceinline__ void bld(float2& v, Rsrc r, unsigned vo, unsigned so) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(vo), static_cast<int>(so), 0);
    v.x = __uint_as_float(w.x);
    v.y = __uint_as_float(w.y);
}
__device__ __forceinline__ void bld(double2& v, Rsrc r, unsigned vo, unsigned so) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(vo), static_cast<int>(so), 0);
    v.x = __hiloint2double(static_cast<int>(w.y), static_cast<int>(w.x));
    v.y = __hiloint2double(static_cast<int>(w.w), static_cast<int>(w.z));
}
// Non-temporal cache policy (bit 1 of the buffer instruction's cache-policy
// operand) for data touched once, so it does not evict the rows neighbouring
// tiles still read: the output stores of applies too large for the
// last-level cache (NT, a kernel instance of its own) and (nt, wave-uniform)
// the per-point data of launches that read them once.  Outputs of smaller
// launches stay cached for the kernel that reads them next.
constexpr int kNt = 2;
// Stores take their whole offset in the vector operand (vo + so, below 2^32:
// a lane's offset kOff = 2^31 plus a plane offset below 2^31 stays beyond
// every buffer, a valid one stays inside): the compiler keeps the z loop's
// plane offset in a vector register, and as the scalar operand it would wrap
// every store in a loop over the lanes' distinct values.
template <bool NT>
__device__ __forceinline__ void bst(Cx<float> v, Rsrc r, unsigned vo, unsigned so) {
    u32x2 w;
    w.x = __float_as_uint(v.re);
    w.y = __float_as_uint(v.im);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, static_cast<int>(vo + so), 0, NT ? kNt : 0);
}
template <bool NT>
__device__ __forceinline__ void bst(Cx<double> v, Rsrc r, unsigned vo, unsigned so) {
    u32x4 w;
    w.x = static_cast<unsigned>(__double2loint(v.re));
    w.y = static_cast<unsigned>(__double2hiint(v.re));
    w.z = static_cast<unsigned>(__double2loint(v.im));
    w.w = static_cast<unsigned>(__double2hiint(v.im));
    __builtin_amdgcn_raw_buffer_store_b128(w, r, static_cast<int>(vo + so), 0, NT ? kNt : 0);
}
__device__ __forceinline__ int bld_u16(Rsrc r, unsigned vo, unsigned so, bool nt = false) {
    return static_cast<int>(nt ? __builtin_amdgcn_raw_buffer_load_b16(r, static_cast<int>(vo), static_cast<int>(so), kNt)
                               : __builtin_amdgcn_raw_buffer_load_b16(r, static_cast<int>(vo), static_cast<int>(so), 0));
}
__device__ __forceinline__ float bld_f32(Rsrc r, unsigned vo, unsigned so, bool nt = false) {
    return __uint_as_float(nt ? __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(vo), static_cast<int>(so), kNt)
                              : __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(vo), static_cast<int>(so), 0));
}

// table entry reads from LDS as 16-byte loads
__device__ __forceinline__ void tab_sm(const TabEntry<float>* t, int e, float (&s)[4], float (&m)[4]) {
    const float4* p = reinterpret_cast<const float4*>(t + e);
    const float4 a = p[0], b = p[1];
    s[0] = a.x; s[1] = a.y; s[2] = a.z; s[3] = a.w;
    m[0] = b.x; m[1] = b.y; m[2] = b.z; m[3] = b.w;
}
__device__ __forceinline__ void tab_sm(const TabEntry<double>* t, int e, double (&s)[4], double (&m)[4]) {
    const double2* p = reinterpret_cast<const double2*>(t + e);
    const double2 a = p[0], b = p[1], c = p[2], d = p[3];
    s[0] = a.x; s[1] = a.y; s[2] = b.x; s[3] = b.y;
    m[0] = c.x; m[1] = c.y; m[2] = d.x; m[3] = d.y;
}
__device__ __forceinline__ void tab_bm(const TabEntry<float>* t, int e, float& b2, float& b3, float (&m)[4]) {
    const float4* p = reinterpret_cast<const float4*>(t + e);
    const float4 b = p[1], c = p[2];
    m[0] = b.x; m[1] = b.y; m[2] = b.z; m[3] = b.w;
    b2 = c.x; b3 = c.y;
}
__device__ __forceinline__ void tab_bm(const TabEntry<double>* t, int e, double& b2, double& b3, double (&m)[4]) {
    const double2* p = reinterpret_cast<const double2*>(t + e);
    const double2 c = p[2], d = p[3], x = p[4];
    m[0] = c.x; m[1] = c.y; m[2] = d.x; m[3] = d.y;
    b2 = x.x; b3 = x.y;
}

// per-point data of one output plane: table index, velocity and (residual /
// Jacobi modes) the right-hand side
template <typename R, int NR>
struct Meta {
    int idx[NR];
    float c[NR];
    typename V2<R>::T b[NR];
};

// plane sums of a box tile: centre, 4-face sum and 4-diagonal sum of u and,
// for the first mass form (MA), of v = k^2 u
template <typename R, int NR, bool MA = false>
struct BoxPlane {
    Cx<R> c[NR], f[NR], e[NR];
    Cx<R> cv[MA ? NR : 1], fv[MA ? NR : 1], ev[MA ? NR : 1];
};

// the rows of one plane a wavefront loads: u, and for the first mass form
// the velocity at the same points
template <typename R, int NL, bool MA>
struct RowSlot {
    typename V2<R>::T u[NL];
    float c[MA ? NL : 1];
};

// k^2 = omega^2 / c^2 at a loaded point (0 where the point lies outside the
// grid: the load returned c = 0 and u = 0 there)
template <typename R>
__device__ __forceinline__ R k2_at(R omega2, float c) {
    const R cr = static_cast<R>(c);
    return c > 0.0f ? omega2 * rcp_of(cr * cr) : R(0);
}

// the arrays of one work item (one right-hand side) as buffer resources
template <typename R, int MODE>
struct ItemBuf {
    const typename V2<R>::T* u;
    unsigned vbytes;          // N * sizeof(complex)
    unsigned plane_b;         // plane * sizeof(complex)
    unsigned plane;
    Rsrc ry, rb, ri, rc;
    __device__ __forceinline__ ItemBuf(const WaveArgs<R>& a, int rhs) {
        const GridData<R>& g = a.g;
        using V = typename V2<R>::T;
        const int64_t ro = static_cast<int64_t>(rhs) * g.N;
        vbytes = static_cast<unsigned>(g.N) * static_cast<unsigned>(sizeof(V));
        plane = static_cast<unsigned>(g.plane);
        plane_b = plane * static_cast<unsigned>(sizeof(V));
        u = a.u + ro;
        ry = rsrc(a.y + ro, vbytes);
        rb = rsrc(MODE == MODE_APPLY ? a.y + ro : a.b + ro, vbytes);
        ri = rsrc(g.idx, static_cast<unsigned>(g.N) * 2u);
        rc = rsrc(g.c, static_cast<unsigned>(g.N) * 4u);
    }
    // plane q of u: offsets of the lanes' rows in ofs; zero outside the grid
    template <int NK>
    __device__ __forceinline__ void load_plane(int q, int nz, const unsigned (&ofs)[NK],
                                               typename V2<R>::T (&L)[NK]) const {
        if (MODE == MODE_JACOBI0) {   // the iterate is zero: nothing to read
#pragma unroll
            for (int k = 0; k < NK; ++k) L[k] = typename V2<R>::T{};
            return;
        }
        const bool in = q >= 0 && q < nz;
        const Rsrc r = rsrc(u, in ? vbytes : 0u);
        const unsigned so = in ? static_cast<unsigned>(q) * plane_b : 0u;
#pragma unroll
        for (int k = 0; k < NK; ++k) bld(L[k], r, ofs[k], so);
    }
    // per-point data of plane q (0 <= q < nz); mo = element offsets of the
    // rows; NTM: non-temporal (each point's data read once by the launch)
    template <int NR, bool ROWC, bool NTM>
    __device__ __forceinline__ void load_meta(int q, const unsigned (&mo)[NR], Meta<R, NR>& M) const {
        const unsigned pe = static_cast<unsigned>(q) * plane;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!ROWC) M.idx[r] = bld_u16(ri, mo[r] * 2u, pe * 2u, NTM);
            M.c[r] = bld_f32(rc, mo[r] * 4u, pe * 4u, NTM);
            if (MODE != MODE_APPLY)
                bld(M.b[r], rb, mo[r] * static_cast<unsigned>(sizeof(typename V2<R>::T)), q * plane_b);
        }
    }
};

// ---------------------------------------------------------------------------
// unstretched-box tile.  BLK = false: one wavefront per tile of RY rows, which
// loads its RY + 2 rows per plane.  BLK = true: the block's BW wavefronts
// (blk_waves) take BW stacked tiles of RY rows; each loads its own RY rows
// (wavefront 0 also the row below the block, the last wavefront the row above)
// and passes them to the others through a two-plane LDS ring, so each row is
// read from memory once per block instead of once per tile that needs it
// (1 + 2/(BW RY) instead of 1 + 2/RY loads per output row), at one barrier per
// plane.
// MA: first consistent-mass form (Sec. 2.1, eq. 8): the mass term of row i
// weighs neighbour j by its own bulk modulus, i.e. the row's mass stencil acts
// on v = k^2 u with k^2 = omega^2 / c_j^2 taken at each loaded point, while
// the stiffness acts on u; the rows' velocities are loaded with u (and v
// shared through the ring beside u).
template <typename R, int MODE, bool SHIFTED, int RY, bool ROWC, bool BLK, bool MA = false, int NT = 0>
__device__ __forceinline__ void box_item(const WaveArgs<R>& a, const TabEntry<R>* tab, const AxisNode<R>* zn,
                                         typename V2<R>::T* ring, int tile, int zc, int rhs, int wave, int lane) {
    using V = typename V2<R>::T;
    constexpr unsigned SV = sizeof(V);
    using Plane = BoxPlane<R, RY, MA>;
    constexpr int NL = BLK ? RY + 1 : RY + 2;   // rows this wavefront loads per plane
    constexpr int BW = blk_waves(sizeof(R) == 8);
    constexpr int KB = BW * RY + 2;             // rows of a block plane in the ring
    const GridData<R>& g = a.g;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int gx = a.px0 + tx * kWaveCols - 1 + lane;
    const bool inx = gx >= 0 && gx < g.nx;
    const bool outx = lane >= 1 && lane <= kWaveCols && gx < a.px0 + a.pw;
    const int gxc = min(max(gx, 0), g.nx - 1);
    const int yb = a.py0 + ty * (BLK ? BW * RY : RY);   // first output row of the tile (block)
    const int y0 = yb + (BLK ? wave * RY : 0);          // first output row of this wavefront
    const int z0 = zc * a.zchunk;
    const int z1 = min(z0 + a.zchunk, g.nz);
    const int yend = a.py0 + a.ph;
    unsigned lo[NL];          // byte offsets of the loaded rows (kOff outside the grid)
    unsigned lc[MA ? NL : 1]; // byte offsets of the loaded rows' velocities (MA)
    unsigned so[RY];          // byte offsets of the stored rows (kOff: no output)
    unsigned mo[RY];          // element offsets of the output rows (clamped, always valid)
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        int yy;
        bool use = true;
        if (BLK) {   // own rows, then the block's halo row (first and last wavefront)
            yy = k < RY ? y0 + k : (wave == 0 ? yb - 1 : yb + BW * RY);
            use = k < RY || wave == 0 || wave == BW - 1;
        } else {
            yy = y0 - 1 + k;
        }
        const bool ok = use && inx && yy >= 0 && yy < g.ny;
        lo[k] = ok ? static_cast<unsigned>(yy * g.nx + gx) * SV : kOff;
        if constexpr (MA) lc[k] = ok ? static_cast<unsigned>(yy * g.nx + gx) * 4u : kOff;
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int yy = y0 + r;
        so[r] = (outx && yy < yend) ? static_cast<unsigned>(yy * g.nx + gx) * SV : kOff;
        mo[r] = static_cast<unsigned>(min(yy, g.ny - 1) * g.nx + gxc);
    }
    const ItemBuf<R, MODE> B_(a, rhs);
    const R sig = g.inv_h2;

    auto output = [&](int zo, const Meta<R, RY>& M, const Plane& A, const Plane& B, const Plane& C)
                      __attribute__((always_inline)) {
        const AxisNode<R> Z = zn[z_slot(zo, g.zlo, g.zhi)];
        const unsigned pso = static_cast<unsigned>(zo) * B_.plane_b;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            R s[4], m[4];
            if (ROWC) {
                const EntryCoef<R> F = g.rowcoef[static_cast<int64_t>(zo) * g.plane + mo[r]];
                s[0] = sig * F.s0; s[1] = sig * F.s1; s[2] = sig * F.s2; s[3] = sig * F.s3;
                m[0] = F.m0; m[1] = F.m1; m[2] = F.m2; m[3] = F.m3;
            } else {
                tab_sm(tab, M.idx[r] - a.tab_lo, s, m);
            }
            const R cvr = static_cast<R>(M.c[r]);
            const R kap = g.omega2 * rcp_of(cvr * cvr);
            Cx<R> acc, diag;
            if (MA && Z.plain) {
                // stiffness on u, mass on v = k^2 u (k^2 already inside v)
                const Cx<R> Fc = B.f[r] + A.c[r] + C.c[r];
                const Cx<R> Ec = B.e[r] + A.f[r] + C.f[r];
                const Cx<R> Co = A.e[r] + C.e[r];
                const Cx<R> Fv = B.fv[r] + A.cv[r] + C.cv[r];
                const Cx<R> Ev = B.ev[r] + A.fv[r] + C.fv[r];
                const Cx<R> Cv = A.ev[r] + C.ev[r];
                Cx<R> st = s[0] * B.c[r];
                rmac(st, s[1], Fc);
                rmac(st, s[2], Ec);
                rmac(st, s[3], Co);
                Cx<R> ms = m[0] * B.cv[r];
                rmac(ms, m[1], Fv);
                rmac(ms, m[2], Ev);
                rmac(ms, m[3], Cv);
                if (SHIFTED) {
                    acc = st;
                    cmac(acc, Cx<R>{g.shift_re, g.shift_im}, ms);
                    diag = Cx<R>{s[0] + kap * g.shift_re * m[0], kap * g.shift_im * m[0]};
                } else {
                    acc = st + ms;
                    diag = Cx<R>{s[0] + kap * m[0], R(0)};
                }
            } else if (Z.plain) {
                const Cx<R> Fc = B.f[r] + A.c[r] + C.c[r];
                const Cx<R> Ec = B.e[r] + A.f[r] + C.f[r];
                const Cx<R> Co = A.e[r] + C.e[r];
                if (SHIFTED) {
                    const R kr = kap * g.shift_re, ks = kap * g.shift_im;
                    const Cx<R> K0{s[0] + kr * m[0], ks * m[0]}, K1{s[1] + kr * m[1], ks * m[1]};
                    const Cx<R> K2{s[2] + kr * m[2], ks * m[2]}, K3{s[3] + kr * m[3], ks * m[3]};
                    acc = K0 * B.c[r];
                    cmac(acc, K1, Fc);
                    cmac(acc, K2, Ec);
                    cmac(acc, K3, Co);
                    diag = K0;
                } else {
                    const R A0 = s[0] + kap * m[0], A1 = s[1] + kap * m[1];
                    const R A2 = s[2] + kap * m[2], A3 = s[3] + kap * m[3];
                    acc = A0 * B.c[r];
                    rmac(acc, A1, Fc);
                    rmac(acc, A2, Ec);
                    rmac(acc, A3, Co);
                    diag = Cx<R>{A0, R(0)};
                }
            } else {
                // z-stretched plane: the in-plane class sums of planes zo - 1,
                // zo, zo + 1 with real weights, then the complex z factors
                const R b2 = s[2] + R(2) * s[3];   // beta2 / h^2
                const R x0 = R(4) * b2 - R(4) * sig, x1 = sig - R(2) * b2;
                Cx<R> Sm = s[1] * A.c[r], Sp = s[1] * C.c[r], S0 = s[1] * B.c[r], SX = x0 * B.c[r];
                rmac(Sm, s[2], A.f[r]); rmac(Sm, s[3], A.e[r]);
                rmac(Sp, s[2], C.f[r]); rmac(Sp, s[3], C.e[r]);
                rmac(S0, s[2], B.f[r]); rmac(S0, s[3], B.e[r]);
                rmac(SX, x1, B.f[r]); rmac(SX, b2, B.e[r]);
                // mass sums: of u (second form, k^2 of the row applied below)
                // or of v = k^2 u (first form)
                const Cx<R>* const Ac = MA ? A.cv : A.c;
                const Cx<R>* const Af = MA ? A.fv : A.f;
                const Cx<R>* const Ae = MA ? A.ev : A.e;
                const Cx<R>* const Bc = MA ? B.cv : B.c;
                const Cx<R>* const Bf = MA ? B.fv : B.f;
                const Cx<R>* const Be = MA ? B.ev : B.e;
                const Cx<R>* const Cc = MA ? C.cv : C.c;
                const Cx<R>* const Cf = MA ? C.fv : C.f;
                const Cx<R>* const Ce = MA ? C.ev : C.e;
                Cx<R> Mm = m[1] * Ac[r], Mp = m[1] * Cc[r], MX = m[0] * Bc[r];
                rmac(Mm, m[2], Af[r]); rmac(Mm, m[3], Ae[r]);
                rmac(Mp, m[2], Cf[r]); rmac(Mp, m[3], Ce[r]);
                rmac(MX, m[1], Bf[r]); rmac(MX, m[2], Be[r]);
                const Cx<R> tm{Z.tm_re, Z.tm_im}, tp{Z.tp_re, Z.tp_im};
                const Cx<R> t0 = -(tm + tp);
                const Cx<R> xz{Z.xi_re, Z.xi_im};
                const Cx<R> um2{R(2) * Z.um_re, R(2) * Z.um_im}, up2{R(2) * Z.up_re, R(2) * Z.up_im};
                Cx<R> st = tm * Sm;
                cmac(st, tp, Sp);
                cmac(st, t0, S0);
                cmac(st, xz, SX);
                Cx<R> ms = um2 * Mm;
                cmac(ms, up2, Mp);
                cmac(ms, xz, MX);
                const R kr = MA ? R(1) : kap;   // first form: k^2 is inside v
                if (SHIFTED) {
                    const Cx<R> kc{kr * g.shift_re, kr * g.shift_im};
                    acc = st;
                    cmac(acc, kc, ms);
                } else {
                    acc = st;
                    rmac(acc, kr, ms);
                }
                if (MODE == MODE_JACOBI || MODE == MODE_JACOBI0) {
                    const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
                    diag = s[1] * t0 + x0 * xz + m[0] * (kc * xz);
                } else {
                    diag = zero<R>();
                }
            }
            V bb{};
            if (MODE != MODE_APPLY) bb = M.b[r];
            bst<NT != 0>(finish<R, MODE>(a.omega_j, acc, diag, B.c[r], bb), B_.ry, so[r], pso);
        }
    };
    // one z step: plane q enters, output plane q - 1 leaves.  Plane q + 2 and
    // the per-point data of plane q + 1 are loaded two steps ahead of their
    // use; past the chunk the last plane is loaded again, so every step issues
    // the same loads and the waits stay exact.
    using Slot = RowSlot<R, NL, MA>;
    // plane q of u (and, MA, of the velocity) into a slot; zero outside the grid
    auto load = [&](int q, Slot& L) __attribute__((always_inline)) {
        B_.load_plane(q, g.nz, lo, L.u);
        if constexpr (MA) {
            const bool in = q >= 0 && q < g.nz;
            const Rsrc r = rsrc(g.c, in ? static_cast<unsigned>(g.N) * 4u : 0u);
            const unsigned sq = in ? static_cast<unsigned>(q) * B_.plane * 4u : 0u;
#pragma unroll
            for (int k = 0; k < NL; ++k) L.c[k] = bld_f32(r, lc[k], sq);
        }
    };
    // sums of one plane's rows (centre, faces, diagonals)
    auto sums = [&](const Cx<R> (&U)[RY + 2], Cx<R>* pc, Cx<R>* pf, Cx<R>* pe) __attribute__((always_inline)) {
        Cx<R> sx[RY + 2];
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) sx[k] = nxt_g<64>(U[k]) + prv_g<64>(U[k]);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            pc[r] = U[r + 1];
            pf[r] = sx[r + 1] + U[r] + U[r + 2];
            pe[r] = sx[r] + sx[r + 2];
        }
    };
    auto step = [&](int q, bool out, const Slot& Lc, Slot& Ln, const Plane& A, const Plane& B, Plane& C,
                    const Meta<R, RY>& Mc, Meta<R, RY>& Mn) __attribute__((always_inline)) {
        load(min(q + 2, z1), Ln);
        B_.template load_meta<RY, ROWC, NT == 2>(min(q + 1, z1 - 1), mo, Mn);
        Cx<R> U[RY + 2];
        Cx<R> Vv[MA ? RY + 2 : 1];
        if constexpr (BLK) {
            // ring[slot][row of the block plane][lane]; slot alternates with q;
            // (MA) the v rows follow the u rows of the slot
            V* pl = ring + ((q & 1) * KB * (MA ? 2 : 1)) * 64;
#pragma unroll
            for (int k = 0; k < RY; ++k) pl[(1 + wave * RY + k) * 64 + lane] = Lc.u[k];
            if (wave == 0) pl[lane] = Lc.u[RY];
            if (wave == BW - 1) pl[(KB - 1) * 64 + lane] = Lc.u[RY];
            if constexpr (MA) {
                V* pv = pl + KB * 64;
                auto kv = [&](int k) {
                    const R k2 = k2_at<R>(g.omega2, Lc.c[k]);
                    V w;
                    w.x = k2 * Lc.u[k].x;
                    w.y = k2 * Lc.u[k].y;
                    return w;
                };
#pragma unroll
                for (int k = 0; k < RY; ++k) pv[(1 + wave * RY + k) * 64 + lane] = kv(k);
                if (wave == 0) pv[lane] = kv(RY);
                if (wave == BW - 1) pv[(KB - 1) * 64 + lane] = kv(RY);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) {
                const V v = pl[(wave * RY + k) * 64 + lane];
                U[k] = Cx<R>{v.x, v.y};
                if constexpr (MA) {
                    const V w = pl[(KB + wave * RY + k) * 64 + lane];
                    Vv[k] = Cx<R>{w.x, w.y};
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) {
                U[k] = Cx<R>{Lc.u[k].x, Lc.u[k].y};
                if constexpr (MA) Vv[k] = k2_at<R>(g.omega2, Lc.c[k]) * U[k];
            }
        }
        sums(U, C.c, C.f, C.e);
        if constexpr (MA) sums(Vv, C.cv, C.fv, C.ev);
        if (out) output(q - 1, Mc, A, B, C);
    };

    // slot k % 3 (k = q - z0 + 1) holds the loads, the plane sums and the
    // per-point data of plane q
    Slot L0, L1, L2;
    Plane P0, P1, P2;
    Meta<R, RY> M0, M1, M2;
    if (BLK) __syncthreads();   // the previous item's last ring reads are done
    load(z0 - 1, L0);
    load(z0, L1);
    // planes z0 - 1 and z0 enter without an output; then one output per step
    step(z0 - 1, false, L0, L2, P1, P2, P0, M2, M1);
    step(z0, false, L1, L0, P2, P0, P1, M0, M2);
    int q = z0 + 1;
    for (;;) {
        step(q, true, L2, L1, P0, P1, P2, M1, M0);
        if (++q > z1) break;
        step(q, true, L0, L2, P1, P2, P0, M2, M1);
        if (++q > z1) break;
        step(q, true, L1, L0, P2, P0, P1, M0, M2);
        if (++q > z1) break;
    }
}

// ---------------------------------------------------------------------------
// Unstretched-box block tile with NB right-hand sides per wavefront (FP32):
// the block's 16 wavefronts take one output row each (62 columns, lanes
// along x) of NB consecutive right-hand sides rhs .. rhs + NB - 1, and share
// their plane rows through a two-plane LDS ring as in box_item<BLK>.  The
// table entry, velocity and coefficients of a point are formed once per
// plane for all NB right-hand sides.
//
// z accumulation: with S(p) = (c, f, e) the centre, face-sum and
// diagonal-sum of plane p at the output column, row (x, y, zo) is
//   out(zo) = K_A(zo) . S(zo - 1) + K_B(zo) . S(zo) + K_C(zo) . S(zo + 1)
// with three coefficient triples per row: in an unstretched plane
// K_A = K_C = (K1, K2, K3), K_B = (K0, K1, K2), K_n = s_n + kappa m_n; in a
// z-stretched plane the complex z factors of the row's node enter (see
// zcoef).  Plane q's step finishes out(q - 1) = P(q - 1) + K_C(q - 1) . S(q)
// and starts P(q) = K_A(q) . S(q - 1) + K_B(q) . S(q), so a right-hand side
// keeps one plane of sums and one partial output, and the loads, per-point
// data and partials rotate with period two (prefetch distance one plane; NB
// right-hand sides keep NB times the bytes of one in flight).
template <typename R>
struct ZCoef {
    Cx<R> a[3], b[3], c[3];   // K_A, K_B, K_C
};

// coefficient triples of one row: table entry (s scaled by 1/h^2, m), kappa
// scaled by the mass factor (kc), and the z node of the row
template <typename R, bool REAL>
__device__ __forceinline__ void zcoef(const R (&s)[4], const R (&m)[4], R sig, Cx<R> kc, const AxisNode<R>& Z,
                                      ZCoef<R>& K) {
    if (Z.plain) {
        Cx<R> k[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) k[n] = REAL ? Cx<R>{s[n] + kc.re * m[n], R(0)}
                                                : Cx<R>{s[n] + kc.re * m[n], kc.im * m[n]};
        K.a[0] = k[1]; K.a[1] = k[2]; K.a[2] = k[3];
        K.b[0] = k[0]; K.b[1] = k[1]; K.b[2] = k[2];
        K.c[0] = k[1]; K.c[1] = k[2]; K.c[2] = k[3];
        return;
    }
    const R b2 = s[2] + R(2) * s[3];
    const R x[3] = {R(4) * b2 - R(4) * sig, sig - R(2) * b2, b2};
    const Cx<R> tm{Z.tm_re, Z.tm_im}, tp{Z.tp_re, Z.tp_im};
    const Cx<R> t0 = -(tm + tp);
    const Cx<R> xz{Z.xi_re, Z.xi_im};
    const Cx<R> um2{R(2) * Z.um_re, R(2) * Z.um_im}, up2{R(2) * Z.up_re, R(2) * Z.up_im};
    const Cx<R> kum = kc * um2, kup = kc * up2, kxz = kc * xz;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        K.a[n] = s[n + 1] * tm + m[n + 1] * kum;
        K.c[n] = s[n + 1] * tp + m[n + 1] * kup;
        K.b[n] = s[n + 1] * t0 + x[n] * xz + m[n] * kxz;
    }
}

// k0 . (c, f, e) with k real (REAL) or complex
template <typename R, bool REAL>
__device__ __forceinline__ Cx<R> dot3(const Cx<R> (&k)[3], Cx<R> c, Cx<R> f, Cx<R> e) {
    if (REAL) {
        Cx<R> r = k[0].re * c;
        rmac(r, k[1].re, f);
        rmac(r, k[2].re, e);
        return r;
    }
    Cx<R> r = k[0] * c;
    cmac(r, k[1], f);
    cmac(r, k[2], e);
    return r;
}

template <typename R, int MODE, bool SHIFTED, bool ROWC, int NB, int NT = 0>
__device__ __forceinline__ void box_item_nb(const WaveArgs<R>& a, const TabEntry<R>* tab, const AxisNode<R>* zn,
                                            typename V2<R>::T* ring, int tile, int zc, int rhs, int wave, int lane) {
    using V = typename V2<R>::T;
    constexpr unsigned SV = sizeof(V);
    constexpr int BW = blk_waves(sizeof(R) == 8);
    constexpr int KB = BW + 2;                 // rows of a block plane in the ring (BW own + 2 halo)
    const GridData<R>& g = a.g;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int nvec = min(NB, a.nrhs - rhs);    // right-hand sides of this item (wave-uniform)
    const int gx = a.px0 + tx * kWaveCols - 1 + lane;
    const bool inx = gx >= 0 && gx < g.nx;
    const bool outx = lane >= 1 && lane <= kWaveCols && gx < a.px0 + a.pw;
    const int gxc = min(max(gx, 0), g.nx - 1);
    const int yb = a.py0 + ty * BW;            // first output row of the block
    const int y0 = yb + wave;                  // this wavefront's output row
    const int yh = wave == 0 ? yb - 1 : yb + BW;   // halo row (first and last wavefront)
    const int z0 = zc * a.zchunk;
    const int z1 = min(z0 + a.zchunk, g.nz);
    const unsigned lo0 = (inx && y0 < g.ny) ? static_cast<unsigned>(y0 * g.nx + gx) * SV : kOff;
    const unsigned lo1 = ((wave == 0 || wave == BW - 1) && inx && yh >= 0 && yh < g.ny)
                             ? static_cast<unsigned>(yh * g.nx + gx) * SV : kOff;
    const unsigned so = (outx && y0 < a.py0 + a.ph) ? static_cast<unsigned>(y0 * g.nx + gx) * SV : kOff;
    const unsigned mo = static_cast<unsigned>(min(y0, g.ny - 1) * g.nx + gxc);
    const unsigned vbytes = static_cast<unsigned>(g.N) * SV;
    const unsigned span = vbytes * static_cast<unsigned>(nvec);
    const unsigned plane = static_cast<unsigned>(g.plane);
    const unsigned plane_b = plane * SV;
    const int64_t ro = static_cast<int64_t>(rhs) * g.N;
    const V* ub = a.u + ro;
    const Rsrc ry = rsrc(a.y + ro, span);
    const Rsrc rb = rsrc(MODE == MODE_APPLY ? a.y + ro : a.b + ro, span);
    const Rsrc ri = rsrc(g.idx, static_cast<unsigned>(g.N) * 2u);
    const Rsrc rc = rsrc(g.c, static_cast<unsigned>(g.N) * 4u);
    const R sig = g.inv_h2;
    const bool real_ok = !SHIFTED;

    // plane q of every right-hand side (own row, halo row); zero outside the grid
    auto load_plane = [&](int q, V (&L)[NB][2]) __attribute__((always_inline)) {
        const bool in = q >= 0 && q < g.nz && MODE != MODE_JACOBI0;
        const Rsrc r = rsrc(ub, in ? span : 0u);
        const unsigned sq = in ? static_cast<unsigned>(q) * plane_b : 0u;
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            if (v < nvec) {
                bld(L[v][0], r, lo0, sq + static_cast<unsigned>(v) * vbytes);
                bld(L[v][1], r, lo1, sq + static_cast<unsigned>(v) * vbytes);
            } else {
                L[v][0] = V{};
                L[v][1] = V{};
            }
        }
    };
    struct PMeta {
        int idx;
        float c;
    };
    auto load_meta = [&](int q, PMeta& M) __attribute__((always_inline)) {
        const unsigned pe = static_cast<unsigned>(q) * plane;
        if (!ROWC) M.idx = bld_u16(ri, mo * 2u, pe * 2u, NT == 2);
        M.c = bld_f32(rc, mo * 4u, pe * 4u, NT == 2);
    };
    auto load_b = [&](int q, V (&Bv)[NB]) __attribute__((always_inline)) {
        if (MODE == MODE_APPLY) return;
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            if (v < nvec) bld(Bv[v], rb, mo * SV, static_cast<unsigned>(q) * plane_b + static_cast<unsigned>(v) * vbytes);
            else Bv[v] = V{};
        }
    };
    // coefficient triples of the row in plane q
    auto coefs = [&](int q, const PMeta& M, ZCoef<R>& K, bool& real) __attribute__((always_inline)) {
        R s[4], m[4];
        if (ROWC) {
            const EntryCoef<R> F = g.rowcoef[static_cast<int64_t>(q) * g.plane + mo];
            s[0] = sig * F.s0; s[1] = sig * F.s1; s[2] = sig * F.s2; s[3] = sig * F.s3;
            m[0] = F.m0; m[1] = F.m1; m[2] = F.m2; m[3] = F.m3;
        } else {
            tab_sm(tab, M.idx - a.tab_lo, s, m);
        }
        const R cvr = static_cast<R>(M.c);
        const R kap = g.omega2 * rcp_of(cvr * cvr);
        const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
        const AxisNode<R>& Z = zn[z_slot(q, g.zlo, g.zhi)];
        real = real_ok && Z.plain;
        if (real) zcoef<R, true>(s, m, sig, kc, Z, K);
        else zcoef<R, false>(s, m, sig, kc, Z, K);
    };

    // per right-hand side: plane sums of the previous plane, partial output of
    // the previous plane's row; shared: that row's K_C and diagonal
    Cx<R> Sc[NB], Sf[NB], Se[NB], P[NB];
    Cx<R> KCp[3], diag_p;
    bool realp = true;
    V L0[NB][2], L1[NB][2];
    PMeta M0, M1;
    V B0[NB], B1[NB];

    // one z step: plane q's sums; finishes out(q - 1) when fin, starts P(q)
    // when q is an output plane.  Loads plane q + 1 and the per-point data of
    // plane q + 1 and right-hand side of plane q.
    auto step = [&](int q, bool fin, bool start, const V (&Lc)[NB][2], V (&Ln)[NB][2], const PMeta& Mc,
                    PMeta& Mn, const V (&Bp)[NB], V (&Bc)[NB]) __attribute__((always_inline)) {
        load_plane(min(q + 1, z1), Ln);
        load_meta(min(q + 1, z1 - 1), Mn);
        load_b(min(max(q, z0), z1 - 1), Bc);
        ZCoef<R> K;
        bool real = true;
        if (start) coefs(q, Mc, K, real);
        V* pl = ring + (q & 1) * (NB * KB * 64);
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            V* pv = pl + v * (KB * 64);
            pv[(1 + wave) * 64 + lane] = Lc[v][0];
            if (wave == 0) pv[lane] = Lc[v][1];
            if (wave == BW - 1) pv[(KB - 1) * 64 + lane] = Lc[v][1];
        }
        __syncthreads();
        const unsigned pso = static_cast<unsigned>(q - 1) * plane_b;
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const V* pv = pl + v * (KB * 64);
            Cx<R> U[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const V w = pv[(wave + k) * 64 + lane];
                U[k] = Cx<R>{w.x, w.y};
            }
            Cx<R> sx[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) sx[k] = nxt_g<64>(U[k]) + prv_g<64>(U[k]);
            const Cx<R> c = U[1], f = sx[1] + U[0] + U[2], e = sx[0] + sx[2];
            if (fin) {
                Cx<R> acc = P[v] + (realp ? dot3<R, true>(KCp, c, f, e) : dot3<R, false>(KCp, c, f, e));
                if (v < nvec)
                    bst<NT != 0>(finish<R, MODE>(a.omega_j, acc, diag_p, Sc[v], Bp[v]), ry,
                        so + static_cast<unsigned>(v) * vbytes, pso);
            }
            if (start) {
                P[v] = real ? dot3<R, true>(K.a, Sc[v], Sf[v], Se[v]) + dot3<R, true>(K.b, c, f, e)
                            : dot3<R, false>(K.a, Sc[v], Sf[v], Se[v]) + dot3<R, false>(K.b, c, f, e);
            }
            Sc[v] = c;
            Sf[v] = f;
            Se[v] = e;
        }
        if (start) {
#pragma unroll
            for (int n = 0; n < 3; ++n) KCp[n] = K.c[n];
            diag_p = K.b[0];
            realp = real;
        }
    };

    if (true) __syncthreads();   // the previous item's last ring reads are done
    // plane z0 - 1 enters (no output row), then planes z0 .. z1: plane q
    // starts row q (q < z1) and finishes row q - 1 (q > z0)
    load_plane(z0 - 1, L0);
    load_meta(z0, M1);
#pragma unroll
    for (int v = 0; v < NB; ++v) B1[v] = V{};
    step(z0 - 1, false, false, L0, L1, M0, M1, B0, B1);   // loads plane z0, meta of z0 (again), b of z0
    int q = z0;
    for (;;) {
        step(q, q > z0, q < z1, L1, L0, M1, M0, B1, B0);
        if (++q > z1) break;
        step(q, q > z0, q < z1, L0, L1, M0, M1, B0, B1);
        if (++q > z1) break;
    }
}

// ---------------------------------------------------------------------------
// PML-frame tile: lanes along x in groups of LW (LW - 2 output columns each,
// halo at both ends), 64 / LW groups stacked along y, RQ rows per lane.  The
// 16-lane groups serve the left / right strips, whose rows are unstretched.
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

// contractions of a frame plane; with the first mass form (MA) the mass ones
// (a, d, e) are also taken of v = k^2 u (av, d, e) while the stiffness keeps a of u
template <typename R, int NR, bool MA = false>
struct FramePlane {
    Cx<R> a[NR], b[NR], c[NR], d[NR], e[NR], u[NR];
    Cx<R> av[MA ? NR : 1];
};

template <typename R, int MODE, bool SHIFTED, int RQ, int LW, bool ROWC, bool MA = false, int NT = 0>
__device__ __forceinline__ void frame_item(const WaveArgs<R>& a, const TabEntry<R>* tab, const AxisNode<R>* zn,
                                           int fr, int ft, int zc, int rhs, int lane) {
    using Plane = FramePlane<R, RQ, MA>;
    using V = typename V2<R>::T;
    constexpr unsigned SV = sizeof(V);
    constexpr bool QPLAIN = LW == 16;   // left / right strips: rows unstretched
    const GridData<R>& g = a.g;
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
    unsigned lo[RQ + 2], so[RQ], mo[RQ];
    unsigned lcv[MA ? RQ + 2 : 1];   // velocity offsets of the loaded rows (MA)
#pragma unroll
    for (int k = 0; k < RQ + 2; ++k) {
        const int qq = q0 - 1 + k;
        const bool ok = inl && qq >= 0 && qq < g.ny;
        lo[k] = ok ? static_cast<unsigned>(qq * g.nx + lc) * SV : kOff;
        if constexpr (MA) lcv[k] = ok ? static_cast<unsigned>(qq * g.nx + lc) * 4u : kOff;
    }
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        const int qq = q0 + r;
        FQ[r] = factors<R>(g.ay[min(qq, g.ny - 1)]);
        xLQ[r] = QPLAIN ? FL.xi : FL.xi * FQ[r].xi;
        so[r] = (outl && qq < y_org + y_ext) ? static_cast<unsigned>(qq * g.nx + lc) * SV : kOff;
        mo[r] = static_cast<unsigned>(min(qq, g.ny - 1) * g.nx + lcc);
    }
    const ItemBuf<R, MODE> B_(a, rhs);
    const R sig = g.inv_h2;

    auto output = [&](int zo, const Meta<R, RQ>& M, const Plane& A, const Plane& B, const Plane& C)
                      __attribute__((always_inline)) {
        const AxisNode<R> Z = zn[z_slot(zo, g.zlo, g.zhi)];
        const bool plainz = Z.plain != 0;
        const Factors<R> FZ = factors<R>(Z);
        const unsigned pso = static_cast<unsigned>(zo) * B_.plane_b;
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            R b2, b3, m[4];
            if (ROWC) {
                const EntryCoef<R> E = g.rowcoef[static_cast<int64_t>(zo) * g.plane + mo[r]];
                b2 = E.beta2; b3 = E.beta3; m[0] = E.m0; m[1] = E.m1; m[2] = E.m2; m[3] = E.m3;
            } else {
                tab_bm(tab, M.idx[r] - a.tab_lo, b2, b3, m);
            }
            const R cvr = static_cast<R>(M.c[r]);
            const R kap = g.omega2 * rcp_of(cvr * cvr);
            Cx<R> PTA = A.a[r], PTB = B.a[r], PTC = C.a[r];
            rmac(PTA, b2, A.b[r]); rmac(PTA, b3, A.c[r]);
            rmac(PTB, b2, B.b[r]); rmac(PTB, b3, B.c[r]);
            rmac(PTC, b2, C.b[r]); rmac(PTC, b3, C.c[r]);
            const R w1 = R(2) * m[1], w2 = R(4) * m[2], w3 = R(8) * m[3];
            // mass contractions: of u (second form) or of v = k^2 u (first form)
            const Cx<R>* const Aa = MA ? A.av : A.a;
            const Cx<R>* const Ba = MA ? B.av : B.a;
            const Cx<R>* const Ca = MA ? C.av : C.a;
            Cx<R> PUA = w1 * Aa[r], PUC = w1 * Ca[r];
            rmac(PUA, w2, A.d[r]); rmac(PUA, w3, A.e[r]);
            rmac(PUC, w2, C.d[r]); rmac(PUC, w3, C.e[r]);
            Cx<R> PXs = B.b[r];
            rmac(PXs, b2, B.c[r]);
            Cx<R> PXm = m[0] * Ba[r];
            rmac(PXm, w1, B.d[r]); rmac(PXm, w2, B.e[r]);
            Cx<R> stiff, mass;
            if (plainz) {   // T_z = (1, -2, 1), X_z = 1, U_z = (1/2, 0, 1/2)
                stiff = PTA + PTC + PXs - R(2) * PTB;
                mass = PXm + R(0.5) * (PUA + PUC);
            } else {
                stiff = FZ.tm * PTA;
                cmac(stiff, FZ.t0, PTB);
                cmac(stiff, FZ.tp, PTC);
                cmac(stiff, FZ.xi, PXs);
                mass = FZ.um * PUA;
                cmac(mass, FZ.up, PUC);
                cmac(mass, FZ.xi, PXm);
            }
            Cx<R> acc = sig * stiff;
            const R kr = MA ? R(1) : kap;   // first form: k^2 is inside v
            if (SHIFTED) {
                cmac(acc, Cx<R>{kr * g.shift_re, kr * g.shift_im}, mass);
            } else {
                rmac(acc, kr, mass);
            }
            Cx<R> diag = zero<R>();
            if (MODE == MODE_JACOBI || MODE == MODE_JACOBI0) {
                const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
                const Factors<R>& Q = FQ[r];
                const Cx<R> ac = xLQ[r];
                const Cx<R> bc = QPLAIN ? FL.t0 + R(-2) * FL.xi : FL.t0 * Q.xi + FL.xi * Q.t0;
                const Cx<R> cc = QPLAIN ? R(-2) * FL.t0 : FL.t0 * Q.t0;
                Cx<R> pc = ac;
                rmac(pc, b2, bc);
                rmac(pc, b3, cc);
                Cx<R> pxs = bc;
                rmac(pxs, b2, cc);
                diag = sig * (FZ.t0 * pc + FZ.xi * pxs) + (m[0] * kc) * (FZ.xi * ac);
            }
            V bb{};
            if (MODE != MODE_APPLY) bb = M.b[r];
            bst<NT != 0>(finish<R, MODE>(a.omega_j, acc, diag, B.u[r], bb), B_.ry, so[r], pso);
        }
    };
    using Slot = RowSlot<R, RQ + 2, MA>;
    auto load = [&](int q, Slot& L) __attribute__((always_inline)) {
        B_.load_plane(q, g.nz, lo, L.u);
        if constexpr (MA) {
            const bool in = q >= 0 && q < g.nz;
            const Rsrc r = rsrc(g.c, in ? static_cast<unsigned>(g.N) * 4u : 0u);
            const unsigned sq = in ? static_cast<unsigned>(q) * B_.plane * 4u : 0u;
#pragma unroll
            for (int k = 0; k < RQ + 2; ++k) L.c[k] = bld_f32(r, lcv[k], sq);
        }
    };
    auto step = [&](int q, bool out, const Slot& Lc, Slot& Ln, const Plane& A, const Plane& B, Plane& C,
                    const Meta<R, RQ>& Mc, Meta<R, RQ>& Mn) __attribute__((always_inline)) {
        load(min(q + 2, z1), Ln);
        B_.template load_meta<RQ, ROWC, NT == 2>(min(q + 1, z1 - 1), mo, Mn);
        Cx<R> U[RQ + 2];
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) U[k] = Cx<R>{Lc.u[k].x, Lc.u[k].y};
        // the mass contractions act on W: u (second form) or v = k^2 u (first)
        Cx<R> W[RQ + 2];
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) W[k] = MA ? k2_at<R>(g.omega2, Lc.c[MA ? k : 0]) * U[k] : U[k];
        Cx<R> RT[RQ + 2], RU[RQ + 2];
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) {
            const Cx<R> vm = prv_g<LW>(U[k]), vp = nxt_g<LW>(U[k]);
            RT[k] = FL.tm * vm + FL.t0 * U[k] + FL.tp * vp;
            const Cx<R> wm = MA ? prv_g<LW>(W[k]) : vm, wp = MA ? nxt_g<LW>(W[k]) : vp;
            RU[k] = FL.um * wm + FL.up * wp;
        }
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            C.u[r] = U[r + 1];
            C.a[r] = xLQ[r] * U[r + 1];
            if constexpr (MA) C.av[r] = xLQ[r] * W[r + 1];
            if (QPLAIN) {   // row factors T = (1, -2, 1), X = 1, U = (1/2, 0, 1/2)
                const Cx<R> ys = U[r] + U[r + 2];
                const Cx<R> ysw = W[r] + W[r + 2];
                C.b[r] = RT[r + 1] + FL.xi * (ys - R(2) * U[r + 1]);
                C.c[r] = RT[r] + RT[r + 2] - R(2) * RT[r + 1];
                C.d[r] = RU[r + 1] + R(0.5) * (FL.xi * ysw);
                C.e[r] = R(0.5) * (RU[r] + RU[r + 2]);
            } else {
                const Factors<R>& Q = FQ[r];
                C.b[r] = Q.xi * RT[r + 1] + FL.xi * (Q.tm * U[r] + Q.t0 * U[r + 1] + Q.tp * U[r + 2]);
                C.c[r] = Q.tm * RT[r] + Q.t0 * RT[r + 1] + Q.tp * RT[r + 2];
                C.d[r] = Q.xi * RU[r + 1] + FL.xi * (Q.um * W[r] + Q.up * W[r + 2]);
                C.e[r] = Q.um * RU[r] + Q.up * RU[r + 2];
            }
        }
        if (out) output(q - 1, Mc, A, B, C);
    };

    // slot k % 3 (k = q - z0 + 1) holds the loads, the plane sums and the
    // per-point data of plane q
    Slot L0, L1, L2;
    Plane P0, P1, P2;
    Meta<R, RQ> M0, M1, M2;
    load(z0 - 1, L0);
    load(z0, L1);
    step(z0 - 1, false, L0, L2, P1, P2, P0, M2, M1);
    step(z0, false, L1, L0, P2, P0, P1, M0, M2);
    int q = z0 + 1;
    for (;;) {
        step(q, true, L2, L1, P0, P1, P2, M1, M0);
        if (++q > z1) break;
        step(q, true, L0, L2, P1, P2, P0, M2, M1);
        if (++q > z1) break;
        step(q, true, L1, L0, P2, P0, P1, M0, M2);
        if (++q > z1) break;
    }
}

// register budget: 4 waves per SIMD (128 VGPRs) for FP32, 2 for FP64.
// NB > 1 (FP32 block tiles, one row per wavefront): box items take NB
// right-hand sides per wavefront (box_item_nb); frame items run their NB
// right-hand sides one after another.
// The body of one block: stage the grid's table slice and z nodes, then
// take work items lb, lb + nb, ... (block granularity; with !BLK each of the
// block's wavefronts takes its own item of the block's group of four).
template <typename R, int MODE, bool SHIFTED, int RY, int RQ, bool ROWC, bool BLK, int NB, bool MA, int NT>
__device__ __forceinline__ void wave27_body(const WaveArgs<R>& a, int nb, int lb, unsigned char* smem_raw) {
    const GridData<R>& g = a.g;
    const int n_tab = ROWC ? 0 : a.n_tab;
    TabEntry<R>* tab = reinterpret_cast<TabEntry<R>*>(smem_raw);
    AxisNode<R>* zn = reinterpret_cast<AxisNode<R>*>(smem_raw + static_cast<size_t>(n_tab) * sizeof(TabEntry<R>));
    const R sig = g.inv_h2;
    for (int t = threadIdx.x; t < n_tab; t += static_cast<int>(blockDim.x)) {
        const EntryCoef<R> E = g.entry[g.fixed ? 0 : a.tab_lo + t];   // fixed weights: one entry everywhere
        TabEntry<R> e;
        e.s[0] = sig * E.s0; e.s[1] = sig * E.s1; e.s[2] = sig * E.s2; e.s[3] = sig * E.s3;
        e.m[0] = E.m0; e.m[1] = E.m1; e.m[2] = E.m2; e.m[3] = E.m3;
        e.b2 = E.s2 + R(2) * E.s3;
        e.b3 = E.s3;
        e.pad0 = e.pad1 = R(0);
        tab[t] = e;
    }
    const int nzl = z_lds_nodes(g.nz, g.zlo, g.zhi);
    for (int t = threadIdx.x; t < nzl; t += static_cast<int>(blockDim.x)) zn[t] = g.az[z_plane(t, g.zlo, g.zhi)];
    // row ring after the table slice and the z nodes, 16-byte aligned (as wave_ring_offset)
    const size_t ring_off = (static_cast<size_t>(n_tab) * sizeof(TabEntry<R>) +
                             static_cast<size_t>(nzl) * sizeof(AxisNode<R>) + 15) & ~static_cast<size_t>(15);
    typename V2<R>::T* ring = reinterpret_cast<typename V2<R>::T*>(smem_raw + ring_off);
    __syncthreads();
    const int wave = uni(static_cast<int>(threadIdx.x) >> 6);
    const int lane = static_cast<int>(threadIdx.x) & 63;
    if (!BLK) {
        const int ntile = a.n_frame + a.n_plain;
        for (int item = lb * (kBlock / 64) + wave; item < a.n_items; item += nb * (kBlock / 64)) {
            // item order: right-hand side fastest, then tile, then z chunk
            // (rhs_outer: tile fastest, then z chunk, then right-hand side)
            const int n_t = ntile * a.nzc;
            const int rhs = a.rhs_outer ? item / n_t : item % a.ngrp;
            const int t = a.rhs_outer ? item % n_t : item / a.ngrp;
            const int tile = t % ntile;
            const int zc = t / ntile;
            if (tile < a.n_frame) {
                int k = 0;
                while (k < 3 && tile >= a.fstart[k + 1]) ++k;
                if (a.flx[k])
                    frame_item<R, MODE, SHIFTED, RQ, 64, ROWC, MA, NT>(a, tab, zn, k, tile - a.fstart[k], zc, rhs, lane);
                else
                    frame_item<R, MODE, SHIFTED, RQ, 16, ROWC, MA, NT>(a, tab, zn, k, tile - a.fstart[k], zc, rhs, lane);
            } else {
                box_item<R, MODE, SHIFTED, RY, ROWC, false, MA, NT>(a, tab, zn, ring, tile - a.n_frame, zc, rhs, wave,
                                                                lane);
            }
        }
    } else {
        // block items: BW frame tiles (one per wavefront) or one box block
        // tile (BW stacked tiles sharing rows through the LDS ring)
        constexpr int BW = blk_waves(sizeof(R) == 8);
        const int nfb = (a.n_frame + BW - 1) / BW;
        const int nbt = nfb + a.n_plain;   // n_plain counts box block tiles here
        for (int bi = lb; bi < a.n_items; bi += nb) {
            // item order: right-hand-side group fastest, then block tile, then z chunk
            // (rhs_outer: block tile fastest, then z chunk, then group)
            const int n_t = nbt * a.nzc;
            const int rhs = (a.rhs_outer ? bi / n_t : bi % a.ngrp) * NB;
            const int t = a.rhs_outer ? bi % n_t : bi / a.ngrp;
            const int bt = t % nbt;
            const int zc = t / nbt;
            if (bt < nfb) {
                const int tile = bt * BW + wave;
                if (tile < a.n_frame) {
                    int k = 0;
                    while (k < 3 && tile >= a.fstart[k + 1]) ++k;
                    const int nv = min(NB, a.nrhs - rhs);
                    for (int v = 0; v < nv; ++v) {
                        if (a.flx[k])
                            frame_item<R, MODE, SHIFTED, RQ, 64, ROWC, MA, NT>(a, tab, zn, k, tile - a.fstart[k], zc, rhs + v,
                                                                       lane);
                        else
                            frame_item<R, MODE, SHIFTED, RQ, 16, ROWC, MA, NT>(a, tab, zn, k, tile - a.fstart[k], zc, rhs + v,
                                                                       lane);
                    }
                }
            } else if constexpr (NB > 1) {
                box_item_nb<R, MODE, SHIFTED, ROWC, NB, NT>(a, tab, zn, ring, bt - nfb, zc, rhs, wave, lane);
            } else {
                box_item<R, MODE, SHIFTED, RY, ROWC, true, MA, NT>(a, tab, zn, ring, bt - nfb, zc, rhs, wave, lane);
            }
        }
    }
}

template <typename R, int MODE, bool SHIFTED, int RY, int RQ, bool ROWC, bool BLK, int NB, bool MA = false,
          int NT = 0>
__global__ __launch_bounds__(BLK ? 64 * blk_waves(sizeof(R) == 8) : kBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
void wave27_kernel(WaveArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // XCD-contiguous block order: block b runs on XCD b % 8; the grid is at
    // most one resident wave per slot and each wave strides over the items
    const int nb = static_cast<int>(gridDim.x);
    const int bx = static_cast<int>(blockIdx.x);
    const int xcd = bx & 7, q8 = nb >> 3, r8 = nb & 7;
    const int lb = xcd * q8 + min(xcd, r8) + (bx >> 3);
    wave27_body<R, MODE, SHIFTED, RY, RQ, ROWC, BLK, NB, MA, NT>(a, nb, lb, smem_raw);
}

// Several grids in one launch (batches of small grids): grid o owns blocks
// [bstart[o], bstart[o + 1]); each block stages its own grid's table slice
// and z nodes and runs the per-wavefront items of that grid.  The arguments
// travel by value in the kernel-argument segment (kWaveBatch grids at most).
constexpr int kWaveBatch = 8;
template <typename R>
struct WaveBatch {
    WaveArgs<R> a[kWaveBatch];
    int bstart[kWaveBatch + 1];
    int n;
};

template <typename R, int MODE, bool SHIFTED, int RY, int RQ, bool ROWC, bool MA>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
void wave27_batch_kernel(WaveBatch<R> B) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int bx = static_cast<int>(blockIdx.x);
    int o = 0;
    while (o + 1 < B.n && bx >= B.bstart[o + 1]) ++o;
    o = uni(o);
    wave27_body<R, MODE, SHIFTED, RY, RQ, ROWC, false, 1, MA, 0>(B.a[o], B.bstart[o + 1] - B.bstart[o],
                                                                     bx - B.bstart[o],
                                                              smem_raw);
}

template <typename R> struct FrameRows;
template <> struct FrameRows<float> { static constexpr int value = 1; };
template <> struct FrameRows<double> { static constexpr int value = 1; };

// blocks of one kernel that fit on the device at once (cached per kernel and
// LDS size; queried on the current device)
inline int resident_blocks(const void* fn, size_t lds, int threads) {
    struct Entry { const void* fn; size_t lds; int dev; int blocks; };
    static thread_local Entry cache[64] = {};
    static thread_local int next = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    for (const Entry& e : cache)
        if (e.fn == fn && e.lds == lds && e.dev == dev) return e.blocks;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int blocks = per_cu * cus;
    cache[next] = Entry{fn, lds, dev, blocks};
    next = (next + 1) % 64;
    return blocks;
}

template <typename R, int MODE, bool SHIFTED, int RY, bool ROWC, bool BLK, int NB, bool MA, int NT>
inline int launch_wave_kn(const WaveArgs<R>& a, hipStream_t s) {
    constexpr int RQ = FrameRows<R>::value;
    const void* fn = reinterpret_cast<const void*>(&wave27_kernel<R, MODE, SHIFTED, RY, RQ, ROWC, BLK, NB, MA, NT>);
    const int n_tab = ROWC ? 0 : a.n_tab;
    const size_t lds = wave_ring_offset(n_tab, z_lds_nodes(a.g.nz, a.g.zlo, a.g.zhi), sizeof(R) == 8) +
                       (BLK ? wave_ring_bytes(RY, NB, sizeof(R) == 8, MA) : 0);
    int blocks = BLK ? a.n_items : (a.n_items + (kBlock / 64) - 1) / (kBlock / 64);
    constexpr int threads = BLK ? 64 * blk_waves(sizeof(R) == 8) : kBlock;
    const int cap = resident_blocks(fn, lds, threads);
    if (cap <= 0) return HELM27_EDEVICE;
    if (blocks > cap) blocks = cap;
    H27_CHECK_HIP(launch(wave27_kernel<R, MODE, SHIFTED, RY, RQ, ROWC, BLK, NB, MA, NT>, dim3(blocks), dim3(threads), lds,
                         s, a));
    return HELM27_OK;
}

// Block-tile applies too large for the last-level cache store their output
// non-temporally, and read their per-point data non-temporally too when
// every point is visited once (NT = 1, 2: kernel instances of their own, so
// the cache policy costs no registers); the other modes' outputs are read
// again by the solver's next kernel
template <typename R, int MODE, bool SHIFTED, int RY, bool ROWC, bool BLK, int NB, bool MA = false>
inline int launch_wave_k(const WaveArgs<R>& a, hipStream_t s) {
    if constexpr (MODE == MODE_APPLY && BLK && !SHIFTED) {
        if (a.nt_store && a.nt_meta) return launch_wave_kn<R, MODE, SHIFTED, RY, ROWC, BLK, NB, MA, 2>(a, s);
        if (a.nt_store) return launch_wave_kn<R, MODE, SHIFTED, RY, ROWC, BLK, NB, MA, 1>(a, s);
    }
    return launch_wave_kn<R, MODE, SHIFTED, RY, ROWC, BLK, NB, MA, 0>(a, s);
}

template <typename R, int MODE, bool SHIFTED, int RY>
inline int launch_wave_ry(const WaveArgs<R>& a, hipStream_t s) {
    if (a.g.mass_a) {   // first mass form: one right-hand side and one row per wavefront
        if constexpr (RY == 1) {
            if (a.nb > 1) return HELM27_EINVAL;
            if (a.blk)
                return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, RY, true, true, 1, true>(a, s)
                                   : launch_wave_k<R, MODE, SHIFTED, RY, false, true, 1, true>(a, s);
            return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, RY, true, false, 1, true>(a, s)
                               : launch_wave_k<R, MODE, SHIFTED, RY, false, false, 1, true>(a, s);
        }
        return HELM27_EINVAL;
    }
    if (a.nb > 1) {   // several right-hand sides per box wavefront: FP32 block tiles, one row
        if constexpr (sizeof(R) == 4 && RY == 1) {
            if (!a.blk) return HELM27_EINVAL;
            if (a.nb == 2)
                return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, 1, true, true, 2>(a, s)
                                   : launch_wave_k<R, MODE, SHIFTED, 1, false, true, 2>(a, s);
            if (a.nb == 4)
                return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, 1, true, true, 4>(a, s)
                                   : launch_wave_k<R, MODE, SHIFTED, 1, false, true, 4>(a, s);
        }
        return HELM27_EINVAL;
    }
    if (a.blk)
        return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, RY, true, true, 1>(a, s)
                           : launch_wave_k<R, MODE, SHIFTED, RY, false, true, 1>(a, s);
    return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, RY, true, false, 1>(a, s)
                       : launch_wave_k<R, MODE, SHIFTED, RY, false, false, 1>(a, s);
}

template <typename R, int MODE, bool SHIFTED>
inline int launch_wave_mode(const WaveArgs<R>& a, int ry, hipStream_t s) {
    switch (ry) {
        case 1: return launch_wave_ry<R, MODE, SHIFTED, 1>(a, s);
        case 2: return launch_wave_ry<R, MODE, SHIFTED, 2>(a, s);
        case 3: return launch_wave_ry<R, MODE, SHIFTED, 3>(a, s);
        case 4: return launch_wave_ry<R, MODE, SHIFTED, 4>(a, s);
        default: return HELM27_EINVAL;
    }
}


// per-mode launchers (one translation unit per mode, kernels_wave_*.hip)
template <typename R, int MODE>
int launch_wave_m(const WaveArgs<R>& a, bool shifted, int ry, hipStream_t s);

}  // namespace h27
