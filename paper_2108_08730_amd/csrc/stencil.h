// Device-side argument block of the 27-point stencil kernels.
#pragma once
#include "cplx.h"
#include "internal.h"

namespace h27 {

enum StencilMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_JACOBI = 2 };

constexpr int kPlainTX = 64;   // plain tile width (one wavefront row along x)
constexpr int kPlainTY = 4;    // thread rows per block
constexpr int kFrameT = 16;    // frame tile edge
constexpr int kBlock = 256;
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
    R shift;                       // beta: mass scaled by (1 + i beta)
};

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

}  // namespace h27
