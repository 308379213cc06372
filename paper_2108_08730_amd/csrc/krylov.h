// Host launchers of the Krylov / multigrid kernels (kernels_krylov.hip).
#pragma once
#include "stencil.h"

namespace h27 {

int fill_zero(void* p, int64_t bytes, hipStream_t s);
int inject_sources(double2* b, int64_t N, const int64_t* d_lin, const double2* d_amp, int nsrc, double h,
                   hipStream_t s);
// d_out[rhs] = ||x[rhs]||_2 (FP64); d_partial holds nrhs * max_blocks doubles
template <typename R>
int norms(const void* x, int64_t N, int nrhs, double* d_partial, int max_blocks, double* d_out, hipStream_t s);
// d_h[rhs * ldh + j] = <V_j[rhs], w[rhs]> for j < J (J <= ldh), and
// d_hsum[...] += the same when d_hsum is not null; d_partial holds
// nrhs * ldh * max_blocks * 2 doubles
// d_selfnrm (optional): also ||w[rhs]||.  d_gate0 / d_gate1 (optional): the
// norms of w before / after a first Gram-Schmidt pass; a right-hand side with
// ||after|| >= ||before|| / sqrt(2) gets h = 0 without reading V (no second
// pass needed).  d_partial holds nrhs * (ldh + 1) * max_blocks * 2 doubles.
template <typename R>
int mdot(const void* V, int64_t vstride, int J, const void* w, int64_t N, int nrhs, double* d_partial, int max_blocks,
         double2* d_h, double2* d_hsum, int ldh, hipStream_t s, double* d_selfnrm = nullptr,
         const double* d_gate0 = nullptr, const double* d_gate1 = nullptr);
// w[rhs] -= sum_{j<J} V_j[rhs] d_hc[rhs * ldh + j]; with d_nrm not null also
// d_nrm[rhs] = ||w_new[rhs]|| (FP64, deterministic two-stage sum).  With the
// gate, a right-hand side that needs no second pass keeps w and gets
// d_nrm = d_gate1.
template <typename R>
int cgs_update(const void* V, int64_t vstride, int J, const double2* d_hc, int ldh, void* w, int64_t N, int nrhs,
               double* d_partial, int max_blocks, double* d_nrm, hipStream_t s, const double* d_gate0 = nullptr,
               const double* d_gate1 = nullptr);
// out = x / nrm (mode 0) or x * nrm (mode 1), per right-hand side; the same
// values also to out2 when it is not null, and dinv * out to yout when dinv is
// not null (dinv: one value per point, shared by the right-hand sides)
template <typename Ri, typename Ro>
int scale_by_norm(const void* x, void* out, int64_t N, int nrhs, const double* d_nrm, int mode, hipStream_t s,
                  void* out2 = nullptr, const void* dinv = nullptr, void* yout = nullptr);
// p[0..n) = 1 (complex)
template <typename R>
int fill_one(void* p, int64_t n, hipStream_t s);
// y[rhs] = dinv * b[rhs] per point: the first damped-Jacobi sweep from a zero
// iterate when dinv = omega D^-1
template <typename R>
int dinv_scale(const void* dinv, const void* b, void* y, int64_t N, int nrhs, hipStream_t s);
template <typename R>
int refine_update(double2* u, const void* e, int64_t N, int nrhs, const double* d_nrm, hipStream_t s);
// x[rhs] (+)= sum_{j<k} V_j[rhs] y[rhs][j]; with dinv also yout = dinv * x
template <typename R>
int combine(const void* V, int64_t vstride, int k, const double2* d_y, int ldy, void* x, int64_t N, int nrhs,
            int accumulate, hipStream_t s, const void* dinv = nullptr, void* yout = nullptr);
template <typename R>
int add_inplace(void* x, const void* y, int64_t n, hipStream_t s);
int givens_init(double2* g, int m, int nrhs, const double* beta, hipStream_t s);
int givens_step(int j, int m, int nrhs, const double2* hcol, int ldh, const double* nrm, double2* H, double* cs,
                double2* sn, double2* g, double* est, hipStream_t s);
int upper_solve(int k, int m, int nrhs, const double2* H, const double2* g, double2* y, int ldy, hipStream_t s);
// full-weighting restriction f -> c; with dinv (coarse grid) also yout = dinv * c
template <typename R>
int mg_restrict(const void* f, int nx, int ny, int nz, void* c, int cx, int cy, int cz, int nrhs, hipStream_t s,
                const void* dinv = nullptr, void* yout = nullptr);
template <typename R>
int mg_prolong_add(const void* c, int cx, int cy, int cz, void* f, int nx, int ny, int nz, int nrhs, hipStream_t s);
int inject_velocity(const float* f, int nx, int ny, float* c, int cx, int cy, int cz, hipStream_t s);

}  // namespace h27
