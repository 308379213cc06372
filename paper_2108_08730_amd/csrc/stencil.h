// Device-side argument block of the 27-point stencil kernels.
#pragma once
#include "cplx.h"
#include "internal.h"

namespace h27 {

// MODE_JACOBI0: the first damped-Jacobi sweep from a zero iterate,
// y = omega D^-1 b (the input vector is not read)
enum StencilMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_JACOBI = 2, MODE_JACOBI0 = 3 };

constexpr int kPlainTX = 64;   // plain tile width (one wavefront row along x)
constexpr int kPlainTY = 4;    // thread rows per block
constexpr int kFrameT = 16;    // frame tile edge
constexpr int kBlock = 256;
// wavefronts per block of the block-tile kernels (variant 2): 16 in FP32
// (the kernels fit 128 registers, so four wavefronts per SIMD and 1024
// threads per block), 8 in FP64 (their 200-odd registers allow two per SIMD);
// taller blocks re-read fewer halo rows (1 + 2 / (waves * RY) loads per row)
constexpr int blk_waves(bool fp64) { return fp64 ? 8 : 16; }
constexpr int kRows = 2;      // plain rows per thread (tile height = kPlainTY * kRows)

template <typename R>
struct GridData {
    int nx, ny, nz;
    int64_t plane, N;
    const float* c;
    const uint16_t* idx;
    const EntryCoef<R>* entry;     // [n_g]
    const EntryCoef<R>* rowcoef;   // [N] (GAm) or null
    int fixed;                     // 1: entry[0] on every row
    const AxisNode<R>* ax;
    const AxisNode<R>* ay;
    const AxisNode<R>* az;
    R omega2;                      // omega^2 (k^2 = omega^2 / c^2)
    R inv_h2;                      // 1 / h^2
    R shift_re, shift_im;          // mass scaled by (shift_re + i shift_im); (1, 0) = physical
    int mass_a;                    // 1: first consistent-mass form (bulk modulus of each neighbour)
    int zlo, zhi;                  // unstretched z planes [zlo, zhi): their nodes are identical
};

// The wavefront kernels stage the z-axis nodes in LDS with the unstretched
// planes' (identical) nodes stored once: nodes 0 .. zlo - 1, one plain node,
// then the planes zhi .. nz - 1.  z_lds_nodes: how many; z_slot: the LDS
// slot of plane q; z_plane: the plane whose node slot t holds.
__host__ __device__ inline int z_lds_nodes(int nz, int zlo, int zhi) {
    return zhi > zlo ? nz - (zhi - zlo - 1) : nz;
}
__host__ __device__ inline int z_slot(int q, int zlo, int zhi) {
    return q < zlo ? q : (q < zhi ? zlo : q - zhi + zlo + (zhi > zlo ? 1 : 0));
}
__host__ __device__ inline int z_plane(int t, int zlo, int zhi) {
    return t < zlo ? t : (zhi > zlo && t == zlo ? zlo : t - zlo - (zhi > zlo ? 1 : 0) + zhi);
}

// Stored coefficients in blocks of 64 rows: entry s of row i sits at
// coef[(i / 64) * 27 * 64 + s * 64 + i % 64], so a wavefront's 64 rows read
// each s as one coalesced 512-byte (FP32) segment and the 27 segments of a
// block are one contiguous stretch of memory; coef_elems(N) entries (N
// rounded up to whole blocks).
__host__ __device__ inline int64_t coef_at(int64_t i, int s) {
    return (i >> 6) * (27 * 64) + static_cast<int64_t>(s) * 64 + (i & 63);
}
inline int64_t coef_elems(int64_t N) { return 27 * ((N + 63) / 64 * 64); }

template <typename R>
struct StencilArgs {
    GridData<R> g;
    // tiling
    int px0, py0, pw, ph;          // plain box
    int ptx;                       // plain tiles along x
    int rows;                      // plain rows per thread (tile height = kPlainTY * rows)
    int fx0[4], fy0[4], fw[4], fh[4], ftx[4], fstart[5];
    int n_plain_blocks;
    int zchunk;
    int nrhs;
    const typename V2<R>::T* u;    // [nrhs][N]
    typename V2<R>::T* y;          // [nrhs][N]
    const typename V2<R>::T* b;    // [nrhs][N] (RESID / JACOBI)
    R omega_j;                     // Jacobi damping
};


// Arguments of the wavefront-per-tile kernel: one wavefront per work item
// (a tile of 62 output columns along its lane axis x RY or RQ rows along the
// other in-plane axis x a z chunk x one right-hand side).  Work items are the
// PML-frame tiles (general complex formula) followed by the unstretched-box
// tiles (lanes along x); the weight-table slice is staged in LDS per block.
template <typename R>
struct WaveArgs {
    GridData<R> g;
    int px0, py0, pw, ph;          // unstretched box
    int ntx, nty, n_plain;         // box tiles along x (62 columns) and y (RY rows)
    int fx0[4], fy0[4], fw[4], fh[4];   // frame rectangles
    int flx[4];                    // 1: lane groups of 64 (62 columns), 0: groups of 16 (14 columns)
    int fnl[4], fnq[4];            // tiles along x and along y
    int fstart[5], n_frame;        // prefix sums of frame tiles
    int nzc, zchunk, nrhs, n_items;
    int blk;                       // 1: box tiles in block items of blk_waves stacked tiles (LDS row ring)
    int nb;                        // right-hand sides per box wavefront (1; 2 or 4 with block tiles, one row)
    int ngrp;                      // right-hand-side groups per tile in the item order (nrhs / nb rounded up)
    int rhs_outer;                 // 1: items ordered tile, z chunk, then right-hand-side group
    int tab_lo, n_tab;             // table slice [tab_lo, tab_lo + n_tab)
    int nt_store;                  // 1: apply output stored non-temporally (vectors larger than the last-level cache)
    int nt_meta;                   // 1: and per-point data (index, velocity) read non-temporally (read once)
    const typename V2<R>::T* u;
    typename V2<R>::T* y;
    const typename V2<R>::T* b;
    R omega_j;
};

constexpr int kWaveCols = 62;      // output columns per wavefront (lanes 1..62)

template <typename R>
int launch_wave(const WaveArgs<R>& a, int mode, bool shifted, int ry, int rq, hipStream_t s);
template <typename R>
int frame_rows();
// apply (MODE_APPLY) of n grids in fused launches of up to 8 grids each; all
// n share the kernel instance: mass scaled or not (attenuation), per-row
// coefficients or the table in LDS, mass form.  Per-wavefront tiles, two box
// rows per wavefront in FP32 (one in FP64 or with the first mass form).
template <typename R>
int launch_wave_batch(const WaveArgs<R>* const* w, int n, bool shifted, bool rowc, bool mass_a, hipStream_t s);
// LDS bytes of the wavefront kernel: the staged weight-table slice (n_tab
// entries; 0 with per-row coefficients) and the z-axis PML nodes
size_t wave_lds_bytes(int n_tab, int nz, bool fp64);
size_t wave_ring_offset(int n_tab, int nz, bool fp64);
// LDS bytes of the block kernel's row ring: two planes of 4 ry + 2 rows per
// right-hand side of a wavefront (nb: 2 or 4 take one row, 6 rows each);
// twice that with the first mass form (v = k^2 u rows beside the u rows)
size_t wave_ring_bytes(int ry, int nb, bool fp64, bool mass_a = false);

}  // namespace h27
