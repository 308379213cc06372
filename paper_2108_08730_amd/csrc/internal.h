// Internal declarations shared by the host sources of libhelm27.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "helm27.h"

#define H27_CHECK_HIP(expr)                                                        \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "helm27: %s failed: %s (%s:%d)\n", #expr,         \
                         hipGetErrorString(e_), __FILE__, __LINE__);               \
            return HELM27_EDEVICE;                                                 \
        }                                                                          \
    } while (0)

namespace h27 {

// Launch recorder: while a GraphRec is installed on the calling thread,
// launch() appends a kernel node (depending on the previous one) to its graph
// instead of launching; otherwise it launches on the stream.  Building the
// graph node by node needs no stream capture, so it is unaffected by what
// other threads do on their streams meanwhile.
struct GraphRec {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;
};
GraphRec*& graph_rec();   // the calling thread's recorder (null: launch eagerly)

template <typename... P, typename... A>
inline hipError_t launch(void (*fn)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s, A&&... a) {
    GraphRec* rec = graph_rec();
    if (!rec) {
        hipLaunchKernelGGL(fn, grid, block, lds, s, std::forward<A>(a)...);
        return hipGetLastError();
    }
    if (rec->err != hipSuccess) return rec->err;
    std::tuple<P...> vals(static_cast<P>(a)...);
    void* ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
    std::apply([&](auto&... v) {
        int k = 0;
        ((ptrs[k++] = static_cast<void*>(&v)), ...);
    }, vals);
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = static_cast<unsigned int>(lds);
    kp.kernelParams = ptrs;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    rec->err = hipGraphAddKernelNode(&node, rec->graph, rec->last ? &rec->last : nullptr, rec->last ? 1 : 0, &kp);
    if (rec->err == hipSuccess) rec->last = node;
    return rec->err;
}

// Per-table-entry coefficients used by the kernels (all dimensionless).
// s0..s3: interior stiffness class values (centre, face, edge, corner) times h^2;
// beta2, beta3: weights of the pairwise / triple products of 1D second
// differences in the tensor form of the stiffness;
// m0..m3: per-point mass weights (centre, face, edge, corner).
template <typename R>
struct EntryCoef {
    R s0, s1, s2, s3;
    R beta2, beta3;
    R m0, m1, m2, m3;
    R pad0, pad1;   // 12 values: 48 B (fp32) / 96 B (fp64), aligned loads
};

// Per-node PML data along one axis (complex values as re/im pairs):
// xi = stretch at the node, tm/tp = 1/xi at the half nodes i-1/2, i+1/2,
// um/up = xi at those half nodes / 2.  plain = 1 when all five are the
// unstretched values (xi = 1 at the node and both half nodes).
template <typename R>
struct AxisNode {
    R xi_re, xi_im;
    R tm_re, tm_im, tp_re, tp_im;
    R um_re, um_im, up_re, up_im;
    int plain;
    int pad;
};

struct Rect { int x0, y0, w, h; };

// Column tiling of one grid for the stencil kernels: the plain box (x and y
// both unstretched) in wide tiles, the frame around it in square tiles.
struct Tiling {
    int plain_x0 = 0, plain_y0 = 0, plain_w = 0, plain_h = 0;
    int n_plain_tiles_x = 0, n_plain_tiles_y = 0;
    Rect frame[4];
    int frame_tiles_x[4], frame_tiles_y[4];
    int n_plain_blocks = 0;     // per z chunk
    int n_frame_blocks = 0;     // per z chunk
    int zchunk = 8, n_zchunks = 1;
};

struct Level;  // multigrid level (solver.cpp)

}  // namespace h27

struct helm27_ctx {
    int device = 0;
    size_t hbm_budget = 0;
    std::mutex mu;
    void* serve = nullptr;   // serving state (serve.cpp)
};

struct helm27_table {
    double g_min = 0, dg = 0;   // first abscissa and step (of G, or of s = 1/G when spacing = 1)
    int n_g = 0;
    int spacing = 0;            // 0: G-uniform, 1: uniform in s = 1/G
    std::vector<double> w7;     // [n_g][7]
    // how it was built (helm27_build_table), so that a wider table can be
    // built the same way; lambda < 0: caller-given weights
    double lambda = -1.0;
    int n_ang = 5, diff_order = 1;
    double angle_step = 10.0;
};

namespace h27 {

// Everything the stencil kernels need about one grid (the fine operator or a
// multigrid level).  Device pointers are owned by the object that made it.
struct GridOp {
    int nx = 0, ny = 0, nz = 0;
    int64_t N = 0;
    double h = 0, omega = 0;
    int npml[3] = {0, 0, 0};
    double R = 1e-3, c_ref = 0;
    // PML layer in physical coordinates (node i at x = i h): unstretched for
    // pml_lo[a] <= x <= pml_hi[a], layer width pml_L[a] (0 = no layer)
    double pml_lo[3] = {0, 0, 0}, pml_hi[3] = {0, 0, 0}, pml_L[3] = {0, 0, 0};
    float* d_c = nullptr;                      // velocity [N]
    uint16_t* d_idx = nullptr;                 // table index [N]
    int n_g = 0;
    int idx_lo = 0, idx_hi = 0;                // range of table indices in use
    int fixed = 0;                             // entry 0 on every row
    void* d_setup = nullptr;                   // one allocation holding the entry and axis arrays below
    EntryCoef<float>* d_entry_f = nullptr;     // [n_g]
    EntryCoef<double>* d_entry_d = nullptr;
    EntryCoef<float>* d_row_f = nullptr;       // GAm: per-row averaged entries [N]
    EntryCoef<double>* d_row_d = nullptr;
    AxisNode<float>* d_ax_f[3] = {nullptr, nullptr, nullptr};
    AxisNode<double>* d_ax_d[3] = {nullptr, nullptr, nullptr};
    int zp_lo = 0, zp_hi = 0;                  // unstretched z planes [zp_lo, zp_hi) (identical nodes)
    Tiling tiling;
    int plain_ry[2] = {2, 1};                  // box rows per wavefront: [fp32, fp64] (1..4)
    int kernel_variant = 0;                    // 0: wavefront-per-tile kernel, 1: LDS-tiled kernel
    int wave_zchunk = 0;                       // z planes per wavefront work item (0: automatic)
    int rhs_block = 0;                         // right-hand sides per box wavefront (FP32 block tiles):
                                               // 0 = automatic (1), 1, 2 or 4
    int mass_a = 0;                            // 1: first consistent-mass form (neighbour bulk modulus)
    double att_re = 1.0, att_im = 0.0;         // attenuation factor of k^2: (1 - i/(2Q))^-2 (1 without)
    int rhs_order = 0;                         // work-item order of a multi-RHS launch: 0 = automatic
                                               // (right-hand side slowest), 1 = fastest, 2 = slowest
    bool auto_tile = true;                     // kernel variant, rows and z chunk chosen per launch from
                                               // the work size; an explicit setting or the tuner clears it
    size_t bytes = 0;
};

// Free every device buffer of a GridOp.
void grid_free(GridOp* g);

}  // namespace h27

struct helm27_op {
    helm27_ctx* ctx = nullptr;
    h27::GridOp g;
    double freq = 0;
    int flags = 0;
    float cmin = 0, cmax = 0;        // velocity range of the model
    int64_t n_clamped = 0;
    double g_min_model = 0, g_max_model = 0;
    void* d_coef_f = nullptr;        // stored: float2[27][N]
    void* d_coef_d = nullptr;        // stored: double2[27][N]
    helm27_table table;              // the table it uses (a copy, or the widened one): weights, axis, fit settings
    void* solver = nullptr;          // solver workspace (solver.cpp)
};

namespace h27 {

// table.cpp
void dispersion_rows(double G, double theta, double phi, double H[5], double* g);
void dispersion_rows_inv(double s, double theta, double phi, double H[5], double* g);
void complete_weights(const double w5[5], double w7[7]);
// Tikhonov table over v_min + i dv (i = 0 .. n_g - 1) with the settings of
// `like` (spacing, lambda, angles, difference order); like must come from
// helm27_build_table
int build_table_like(const helm27_table* like, double v_min, int n_g, helm27_table** out);

// op.cpp
int op_build(helm27_ctx* ctx, const double* w7, int n_g, double g_min, double dg,
             const float* vel, int nx, int ny, int nz, double h, double freq, double omega_shift,
             const helm27_pml* pml, int flags, helm27_op** out);
int op_create(helm27_ctx* ctx, const helm27_table* t, const float* vel, int nx, int ny, int nz, double h,
              double freq, const helm27_pml* pml, int flags, hipStream_t stream, helm27_op** out);
// solver.cpp: drop the solver's Krylov workspace (keeps the multigrid hierarchy)
void solver_trim(helm27_op* op);
// device bytes a solve of nrhs right-hand sides would allocate (estimate)
size_t solve_footprint(int64_t N, int nrhs, int restart, int precision, int levels);
void make_tiling(int nx, int ny, const int plain_lo[2], const int plain_hi[2], Tiling* t, int zchunk, int nz);
void axis_nodes(int n, double h, double x_lo, double x_hi, double L, double omega, double c_ref, double R,
                std::vector<AxisNode<double>>* out);
int grid_setup(GridOp* g, const double* w7, int n_g, int fixed);
int host_index(float c, double fh, double gmin, double dg, int n_g, int invg);
// the smallest range on table t's axis grid (v_min - k dv .. v_max + k' dv)
// that covers abscissae need_lo .. need_hi, within the axis' domain (v > 0 on
// the G axis, v >= 0 on the 1/G axis): its first abscissa and entry count
// (ERANGE beyond 65535 entries)
int widen_range(const helm27_table* t, double need_lo, double need_hi, double* v_min, int* n_g);

// kernels (kernels_*.hip): host-side launchers
// d_counts: 4 entries, initialised by the caller to {0, 0, bits of +inf, 0}:
// clamped points, invalid velocities, min / max bit pattern of the valid ones
// look up this device's scratch array of the no-allocation index selection
// (the device must be current)
int noalloc_init(int device);
int launch_select_index(const float* c, uint16_t* idx, int64_t N, double fh, double gmin, double dg,
                        int n_g, int invg, unsigned long long* d_counts, hipStream_t s);
// y = A u (MODE_APPLY), y = b - A u (MODE_RESID), y = u + omega_j D^-1 (b - A u)
// (MODE_JACOBI) or y = omega_j D^-1 b (MODE_JACOBI0, u not read; wavefront
// kernel only) with A's mass scaled by (shift_re + i shift_im); (1, 0) is the
// physical operator.  R = float | double.
template <typename R>
int launch_stencil(const GridOp& g, int mode, double shift_re, double shift_im, const void* u, void* y,
                   const void* b, double omega_j, int nrhs, hipStream_t s);
// y_i = A_i u_i (physical operators) for n grids in fused launches; every
// grid must be eligible for the wavefront kernel (EINVAL otherwise)
template <typename R>
int launch_stencil_batch(const GridOp* const* g, int n, const void* const* u, void* const* y, const int* nrhs,
                         hipStream_t s);
// whether launch_stencil runs the wavefront kernel on this grid (which also
// provides the zero-iterate Jacobi mode)
bool stencil_wave_path(const GridOp& g, bool fp64);
template <typename R>
int launch_fill_stored(const GridOp& g, void* coef, double shift_re, double shift_im, hipStream_t s);
template <typename R>
int launch_apply_stored(const GridOp& g, const void* coef, const void* u, void* y, int nrhs,
                        hipStream_t s);
template <typename R>
int launch_gam_average(const GridOp& g, EntryCoef<R>* rowcoef, hipStream_t s);
// y = A^T u, or y = b - A^T u with b, from the stored coefficients
template <typename R>
int launch_apply_stored_t(const GridOp& g, const void* coef, const void* u, void* y, const void* b, int nrhs,
                          hipStream_t s);

}  // namespace h27
