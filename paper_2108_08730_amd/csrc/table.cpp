// Weight table of the wavelength-adaptive stencil (host, FP64).
//
// Dispersion analysis of Sec. 2.2: a plane wave of G grid points per
// wavelength in direction (theta, phi) has normalised phase velocity
//   v~ = G / (sqrt(2 J) pi) sqrt(Q),
//   Q = w_s1 (3 - C) + w_s2/3 (6 - C - B) + w_s3/2 (3 - 3A + B - C),
//   J = w_m0 + 2 w_m1 C + 4 w_m2 B + 8 w_m3 A,
// with A, B, C the product / pair-sum / sum of the three directional cosines.
// v~ = 1 is linear in the five free weights once w_s3 = 1 - w_s1 - w_s2 and
// w_m3 = (1 - w_m0 - 6 w_m1 - 12 w_m2)/8 are eliminated.  The adaptive table
// solves, over the G grid, the Tikhonov problem
//   min ||H w - g||^2 + lambda ||D P w||^2
// where H is block diagonal (one block of plane-wave rows per G) and D P takes
// first (or second) differences of each weight along G.
//
// Solver: with the unknowns ordered G-major the stacked matrix [H; sqrt(lambda)
// D P] is banded (every row lives in a window of 5 (order+1) columns), so it is
// reduced row by row with Givens rotations into a banded upper-triangular R,
// then back-substituted.  Orthogonal reduction keeps the full accuracy of the
// least-squares solution (the normal equations would square a condition number
// of ~1e11).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

namespace h27 {

void dispersion_rows(double G, double theta, double phi, double H[5], double* g) {
    const double pi = 3.14159265358979323846;
    const double ca = std::cos(2.0 * pi * std::cos(phi) * std::cos(theta) / G);
    const double cb = std::cos(2.0 * pi * std::cos(phi) * std::sin(theta) / G);
    const double cc = std::cos(2.0 * pi * std::sin(phi) / G);
    const double A = ca * cb * cc;
    const double B = ca * cb + ca * cc + cb * cc;
    const double C = ca + cb + cc;
    const double k2 = 2.0 * pi * pi / (G * G);
    // coefficient of w_s1 and w_s2 in Q after eliminating w_s3
    H[0] = 0.5 * (3.0 + 3.0 * A - B - C);
    H[1] = (3.0 + 9.0 * A - 5.0 * B + C) / 6.0;
    // -k2 times the coefficient of w_m0, w_m1, w_m2 in J after eliminating w_m3
    H[2] = k2 * (A - 1.0);
    H[3] = k2 * (6.0 * A - 2.0 * C);
    H[4] = k2 * (12.0 * A - 4.0 * B);
    *g = k2 * A - 0.5 * (3.0 - 3.0 * A + B - C);
}

// The same rows as functions of s = 1/G (the paper's 1/G table axis): phases
// 2 pi s n_a and k2 = 2 pi^2 s^2, so s = 0 (G infinite) gives zero rows.
void dispersion_rows_inv(double s, double theta, double phi, double H[5], double* g) {
    const double pi = 3.14159265358979323846;
    const double ca = std::cos(2.0 * pi * std::cos(phi) * std::cos(theta) * s);
    const double cb = std::cos(2.0 * pi * std::cos(phi) * std::sin(theta) * s);
    const double cc = std::cos(2.0 * pi * std::sin(phi) * s);
    const double A = ca * cb * cc;
    const double B = ca * cb + ca * cc + cb * cc;
    const double C = ca + cb + cc;
    const double k2 = 2.0 * pi * pi * s * s;
    H[0] = 0.5 * (3.0 + 3.0 * A - B - C);
    H[1] = (3.0 + 9.0 * A - 5.0 * B + C) / 6.0;
    H[2] = k2 * (A - 1.0);
    H[3] = k2 * (6.0 * A - 2.0 * C);
    H[4] = k2 * (12.0 * A - 4.0 * B);
    *g = k2 * A - 0.5 * (3.0 - 3.0 * A + B - C);
}

void complete_weights(const double w5[5], double w7[7]) {
    w7[0] = w5[0];
    w7[1] = w5[1];
    w7[2] = 1.0 - w5[0] - w5[1];
    w7[3] = w5[2];
    w7[4] = w5[3];
    w7[5] = w5[4];
    w7[6] = (1.0 - w5[2] - 6.0 * w5[3] - 12.0 * w5[4]) / 8.0;
}

namespace {

// Banded least squares by Givens rotations.  Columns 0..n-1, every added row
// has its nonzeros in [c0, c0 + bw).  R is stored row-wise: R[j][k] is the
// entry (j, j + k), k < bw.
class BandedLS {
  public:
    static constexpr int kMaxBw = 16;   // 5 weights x (difference order + 1) <= 15
    BandedLS(int n, int bw) : n_(n), bw_(bw), R_(static_cast<size_t>(n) * bw, 0.0), qtb_(n, 0.0), filled_(n, 0) {}

    // Add the row (vals[0..bw) at columns c0..c0+bw) with right-hand side rhs.
    void add_row(int c0, const double* vals, double rhs) {
        double r[kMaxBw];
        for (int k = 0; k < bw_; ++k) r[k] = vals[k];
        double b = rhs;
        int off = c0;  // column of r[0]
        for (int j = off; j < n_; ++j) {
            // r currently covers columns [off, off + bw); shift so r[0] is column j
            const int sh = j - off;
            if (sh > 0) {
                for (int k = 0; k < bw_; ++k) r[k] = (k + sh < bw_) ? r[k + sh] : 0.0;
                off = j;
            }
            const double x = r[0];
            if (x == 0.0) {
                bool any = false;
                for (int k = 1; k < bw_; ++k) any = any || r[k] != 0.0;
                if (!any) return;  // row fully absorbed
                continue;
            }
            double* Rj = &R_[static_cast<size_t>(j) * bw_];
            if (!filled_[j]) {
                for (int k = 0; k < bw_; ++k) Rj[k] = r[k];
                qtb_[j] = b;
                filled_[j] = 1;
                return;
            }
            const double a = Rj[0];
            double c, s, rr;
            if (std::fabs(x) > std::fabs(a)) {
                const double t = a / x;
                rr = std::fabs(x) * std::sqrt(1.0 + t * t);
                c = a / rr;
                s = x / rr;
            } else {
                const double t = x / a;
                rr = std::fabs(a) * std::sqrt(1.0 + t * t);
                c = a / rr;
                s = x / rr;
            }
            for (int k = 0; k < bw_; ++k) {
                const double p = Rj[k], q = r[k];
                Rj[k] = c * p + s * q;
                r[k] = -s * p + c * q;
            }
            const double pb = qtb_[j];
            qtb_[j] = c * pb + s * b;
            b = -s * pb + c * b;
            r[0] = 0.0;
        }
    }

    // Back substitution; returns false if R is singular.
    bool solve(std::vector<double>* x) const {
        x->assign(n_, 0.0);
        for (int j = n_ - 1; j >= 0; --j) {
            const double* Rj = &R_[static_cast<size_t>(j) * bw_];
            if (!filled_[j] || Rj[0] == 0.0) return false;
            double s = qtb_[j];
            for (int k = 1; k < bw_ && j + k < n_; ++k) s -= Rj[k] * (*x)[j + k];
            (*x)[j] = s / Rj[0];
        }
        return true;
    }

  private:
    int n_, bw_;
    std::vector<double> R_, qtb_;
    std::vector<char> filled_;
};

// Minimum-norm least squares for a small dense m x n system (row-major A) by
// one-sided Jacobi SVD: the fixed-weight fits are rank deficient (every row of
// the dispersion system is a combination of 1, A, B, C), so their solution is
// the pseudo-inverse one.
bool minnorm_ls(std::vector<double> A, const std::vector<double>& b, int m, int n, double* x) {
    std::vector<double> V(static_cast<size_t>(n) * n, 0.0);
    for (int j = 0; j < n; ++j) V[j * n + j] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double a = 0, bb = 0, c = 0;
                for (int i = 0; i < m; ++i) {
                    const double ap = A[i * n + p], aq = A[i * n + q];
                    a += ap * ap;
                    bb += aq * aq;
                    c += ap * aq;
                }
                if (c == 0.0) continue;
                off = std::max(off, std::fabs(c) / std::sqrt(a * bb));
                const double zeta = (bb - a) / (2.0 * c);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < m; ++i) {
                    const double ap = A[i * n + p], aq = A[i * n + q];
                    A[i * n + p] = cs * ap - sn * aq;
                    A[i * n + q] = sn * ap + cs * aq;
                }
                for (int i = 0; i < n; ++i) {
                    const double vp = V[i * n + p], vq = V[i * n + q];
                    V[i * n + p] = cs * vp - sn * vq;
                    V[i * n + q] = sn * vp + cs * vq;
                }
            }
        if (off < 1e-15) break;
    }
    std::vector<double> sig(n);
    double smax = 0;
    for (int j = 0; j < n; ++j) {
        double s2 = 0;
        for (int i = 0; i < m; ++i) s2 += A[i * n + j] * A[i * n + j];
        sig[j] = std::sqrt(s2);
        smax = std::max(smax, sig[j]);
    }
    if (!(smax > 0)) return false;
    // rank decision: singular values below 1e-10 of the largest are taken as zero
    const double tol = smax * 1e-10;
    for (int k = 0; k < n; ++k) x[k] = 0.0;
    for (int j = 0; j < n; ++j) {
        if (sig[j] <= tol) continue;
        double ub = 0;  // u_j^T b with u_j = A[:, j] / sig_j
        for (int i = 0; i < m; ++i) ub += A[i * n + j] * b[i];
        const double coef = ub / (sig[j] * sig[j]);
        for (int k = 0; k < n; ++k) x[k] += coef * V[k * n + j];
    }
    return true;
}

}  // namespace
}  // namespace h27

using namespace h27;

// In-place Householder QR of a dense m x 5 block (row-major A) applied to b
// as well: on return rows 0..min(m,5)-1 of A hold the upper triangle R and
// b[0..) the first entries of Q^T b.  Returns the number of triangle rows.
static int householder_rows(double* A, double* b, int m) {
    const int n = 5, nk = m < n ? m : n;
    for (int k = 0; k < nk; ++k) {
        double nrm2 = 0.0;
        for (int i = k; i < m; ++i) nrm2 += A[5 * i + k] * A[5 * i + k];
        const double nrm = std::sqrt(nrm2);
        if (nrm == 0.0) continue;
        const double akk = A[5 * k + k];
        const double alpha = akk > 0 ? -nrm : nrm;   // the new diagonal, no cancellation
        // v = x - alpha e_k, stored over column k below the diagonal; v^T v = 2 nrm (nrm + |akk|)
        const double v0 = akk - alpha;
        const double vtv = 2.0 * nrm * (nrm + std::fabs(akk));
        for (int j = k + 1; j < n; ++j) {
            double d = v0 * A[5 * k + j];
            for (int i = k + 1; i < m; ++i) d += A[5 * i + k] * A[5 * i + j];
            const double f = 2.0 * d / vtv;
            A[5 * k + j] -= f * v0;
            for (int i = k + 1; i < m; ++i) A[5 * i + j] -= f * A[5 * i + k];
        }
        double d = v0 * b[k];
        for (int i = k + 1; i < m; ++i) d += A[5 * i + k] * b[i];
        const double f = 2.0 * d / vtv;
        b[k] -= f * v0;
        for (int i = k + 1; i < m; ++i) b[i] -= f * A[5 * i + k];
        A[5 * k + k] = alpha;
        for (int i = k + 1; i < m; ++i) A[5 * i + k] = 0.0;
    }
    return nk;
}

namespace h27 {

// the table over g_min + i dg, i < n_g (the abscissa is G, or s = 1/G when
// spacing = 1), with the given fit settings
static int build_table_impl(double g_min, int n_g, double dg, double lambda, int spacing, int n_ang, double step,
                            int order, helm27_table** out) {
    if (order == 2 && n_g < 3 && lambda > 0) return HELM27_EINVAL;
    if (spacing == 1 && lambda == 0.0) return HELM27_EINVAL;   // the decoupled fits need the G axis
    auto rows = [spacing](double v, double th, double ph, double* H, double* g) {
        if (spacing == 1) dispersion_rows_inv(v, th, ph, H, g);
        else dispersion_rows(v, th, ph, H, g);
    };
    auto stamp = [&](helm27_table* t) {
        t->g_min = g_min;
        t->dg = dg;
        t->n_g = n_g;
        t->spacing = spacing;
        t->lambda = lambda;
        t->n_ang = n_ang;
        t->angle_step = step;
        t->diff_order = order;
    };
    const double pi = 3.14159265358979323846;
    std::vector<double> ang(n_ang);
    for (int k = 0; k < n_ang; ++k) ang[k] = k * step * pi / 180.0;

    if (lambda == 0.0) {
        // no smoothing: each G is its own (rank-deficient) problem
        helm27_table* t = new (std::nothrow) helm27_table;
        if (!t) return HELM27_ENOMEM;
        stamp(t);
        t->w7.resize(static_cast<size_t>(n_g) * 7);
        const int m = n_ang * n_ang;
        for (int i = 0; i < n_g; ++i) {
            std::vector<double> A(static_cast<size_t>(m) * 5), b(m);
            int r = 0;
            for (int jp = 0; jp < n_ang; ++jp)
                for (int jt = 0; jt < n_ang; ++jt, ++r) dispersion_rows(g_min + i * dg, ang[jt], ang[jp], &A[5 * r], &b[r]);
            double w5[5];
            if (!minnorm_ls(A, b, m, 5, w5)) {
                delete t;
                return HELM27_ENUMERIC;
            }
            complete_weights(w5, &t->w7[7 * i]);
        }
        *out = t;
        return HELM27_OK;
    }
    const int n = 5 * n_g;
    const int bw = 5 * (order + 1);
    BandedLS ls(n, bw);
    std::vector<double> row(bw);
    const double sl = std::sqrt(lambda);
    // Each G block's dispersion rows touch only its own five columns: they
    // are reduced to a 5 x 5 triangle (and Q^T b) by Householder reflections
    // first; an orthogonal transformation leaves the least-squares solution
    // unchanged, and the banded factorisation then absorbs 5 rows instead of
    // n_ang^2.  The blocks are independent, so their reductions run on a few
    // host threads (each block's arithmetic is the same on any thread).
    const int m_ang = n_ang * n_ang;
    std::vector<double> Rt(static_cast<size_t>(n_g) * 25), qt(static_cast<size_t>(n_g) * 5);
    std::vector<int> nkb(n_g);
    auto reduce_blocks = [&](int i0, int i1) {
        std::vector<double> Ab(static_cast<size_t>(m_ang) * 5), bb(m_ang);
        for (int i = i0; i < i1; ++i) {
            const double G = g_min + i * dg;
            int r = 0;
            for (int jp = 0; jp < n_ang; ++jp)
                for (int jt = 0; jt < n_ang; ++jt, ++r) rows(G, ang[jt], ang[jp], &Ab[5 * r], &bb[r]);
            const int nk = householder_rows(Ab.data(), bb.data(), m_ang);
            nkb[i] = nk;
            for (int k = 0; k < nk; ++k) {
                for (int l = 0; l < 5; ++l) Rt[25 * static_cast<size_t>(i) + 5 * k + l] = Ab[5 * k + l];
                qt[5 * static_cast<size_t>(i) + k] = bb[k];
            }
        }
    };
    {
        const unsigned hw = std::thread::hardware_concurrency();
        const int nt = std::max(1, std::min({static_cast<int>(hw ? hw : 1), 8, n_g / 64}));
        std::vector<std::thread> pool;
        const int per = (n_g + nt - 1) / nt;
        try {
            for (int t = 1; t < nt; ++t) pool.emplace_back(reduce_blocks, std::min(n_g, t * per), std::min(n_g, (t + 1) * per));
        } catch (...) {
            for (std::thread& th : pool) th.join();
            return HELM27_ENOMEM;
        }
        reduce_blocks(0, std::min(n_g, per));
        for (std::thread& th : pool) th.join();
    }
    for (int i = 0; i < n_g; ++i) {
        for (int k = 0; k < nkb[i]; ++k) {
            std::fill(row.begin(), row.end(), 0.0);
            for (int l = k; l < 5; ++l) row[l - k] = Rt[25 * static_cast<size_t>(i) + 5 * k + l];
            ls.add_row(5 * i + k, row.data(), qt[5 * static_cast<size_t>(i) + k]);
        }
        // smoothing rows whose first column lies in block i
        if (lambda > 0 && i + order < n_g) {
            for (int l = 0; l < 5; ++l) {
                std::fill(row.begin(), row.end(), 0.0);
                if (order == 1) {
                    row[0] = -sl;
                    row[5] = sl;
                } else {
                    row[0] = sl;
                    row[5] = -2.0 * sl;
                    row[10] = sl;
                }
                ls.add_row(5 * i + l, row.data(), 0.0);
            }
        }
    }
    std::vector<double> w;
    if (!ls.solve(&w)) return HELM27_ENUMERIC;
    helm27_table* t = new (std::nothrow) helm27_table;
    if (!t) return HELM27_ENOMEM;
    stamp(t);
    t->w7.resize(static_cast<size_t>(n_g) * 7);
    for (int i = 0; i < n_g; ++i) complete_weights(&w[5 * i], &t->w7[7 * i]);
    *out = t;
    return HELM27_OK;
}

int build_table_like(const helm27_table* like, double v_min, int n_g, helm27_table** out) {
    if (!like || !out || like->lambda < 0 || n_g < 1 || n_g > 65535) return HELM27_EINVAL;
    return build_table_impl(v_min, n_g, like->dg, like->lambda, like->spacing, like->n_ang, like->angle_step,
                            like->diff_order, out);
}

}  // namespace h27

extern "C" int helm27_build_table(helm27_ctx* ctx, double g_min, double g_max, double dg, double lambda,
                                  const helm27_table_opts* opts, helm27_table** out) {
    (void)ctx;
    int n_ang = 5, order = 1, spacing = HELM27_SPACING_G;
    double step = 10.0;
    if (opts) {
        if (opts->n_angles > 0) n_ang = opts->n_angles;
        if (opts->angle_step_deg > 0) step = opts->angle_step_deg;
        if (opts->diff_order == 1 || opts->diff_order == 2) order = opts->diff_order;
        else if (opts->diff_order != 0) return HELM27_EINVAL;
        if (opts->spacing == HELM27_SPACING_G || opts->spacing == HELM27_SPACING_INVG) spacing = opts->spacing;
        else return HELM27_EINVAL;
    }
    const bool lo_ok = spacing == HELM27_SPACING_G ? g_min > 0 : g_min >= 0;
    if (!out || !lo_ok || !(dg > 0) || !(g_max >= g_min) || !(lambda >= 0) || !std::isfinite(g_max))
        return HELM27_EINVAL;
    const double nn = std::round((g_max - g_min) / dg) + 1.0;
    if (nn > 65535.0) return HELM27_EINVAL;
    return h27::build_table_impl(g_min, static_cast<int>(nn), dg, lambda, spacing, n_ang, step, order, out);
}

extern "C" int helm27_table_from_weights(helm27_ctx* ctx, int spacing, double g_min, double dg, int n_g,
                                         const double* w5, helm27_table** out) {
    (void)ctx;
    if (!out || !w5 || n_g <= 0 || n_g > 65535 || !(dg > 0) || !std::isfinite(g_min) ||
        (spacing != HELM27_SPACING_G && spacing != HELM27_SPACING_INVG) ||
        (spacing == HELM27_SPACING_INVG && g_min < 0))
        return HELM27_EINVAL;
    helm27_table* t = new (std::nothrow) helm27_table;
    if (!t) return HELM27_ENOMEM;
    t->g_min = g_min;
    t->dg = dg;
    t->n_g = n_g;
    t->spacing = spacing;
    t->w7.resize(static_cast<size_t>(n_g) * 7);
    for (int i = 0; i < n_g; ++i) {
        for (int k = 0; k < 5; ++k)
            if (!std::isfinite(w5[5 * i + k])) {
                delete t;
                return HELM27_EINVAL;
            }
        complete_weights(&w5[5 * i], &t->w7[7 * i]);
    }
    *out = t;
    return HELM27_OK;
}

extern "C" int helm27_table_weights(const helm27_table* t, double* w7, int* n_g, double* g_min, double* dg) {
    if (!t) return HELM27_EINVAL;
    if (w7) std::memcpy(w7, t->w7.data(), t->w7.size() * sizeof(double));
    if (n_g) *n_g = t->n_g;
    if (g_min) *g_min = t->g_min;
    if (dg) *dg = t->dg;
    return HELM27_OK;
}

extern "C" int helm27_table_axis(const helm27_table* t, int* spacing, double* v_min, double* dv, int* n_g) {
    if (!t) return HELM27_EINVAL;
    if (spacing) *spacing = t->spacing;
    if (v_min) *v_min = t->g_min;
    if (dv) *dv = t->dg;
    if (n_g) *n_g = t->n_g;
    return HELM27_OK;
}

extern "C" void helm27_table_destroy(helm27_table* t) { delete t; }

extern "C" int helm27_fit_fixed(helm27_ctx* ctx, const double* g_list, int n_list, const helm27_table_opts* opts,
                                const double* w5_near, helm27_table** out) {
    (void)ctx;
    if (!out || !g_list || n_list <= 0) return HELM27_EINVAL;
    int n_ang = 5;
    double step = 10.0;
    if (opts) {
        if (opts->n_angles > 0) n_ang = opts->n_angles;
        if (opts->angle_step_deg > 0) step = opts->angle_step_deg;
    }
    const double pi = 3.14159265358979323846;
    const int m = n_list * n_ang * n_ang;
    std::vector<double> A(static_cast<size_t>(m) * 5), b(m);
    int r = 0;
    for (int l = 0; l < n_list; ++l) {
        if (!(g_list[l] > 0)) return HELM27_EINVAL;
        for (int jp = 0; jp < n_ang; ++jp)
            for (int jt = 0; jt < n_ang; ++jt, ++r)
                dispersion_rows(g_list[l], jt * step * pi / 180.0, jp * step * pi / 180.0, &A[5 * r], &b[r]);
    }
    // least-squares solution closest to w5_near (minimum norm without it):
    // near + the minimum-norm solution of A dw = b - A near
    double w0[5] = {0, 0, 0, 0, 0};
    if (w5_near)
        for (int k = 0; k < 5; ++k) {
            if (!std::isfinite(w5_near[k])) return HELM27_EINVAL;
            w0[k] = w5_near[k];
        }
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < 5; ++k) b[i] -= A[5 * static_cast<size_t>(i) + k] * w0[k];
    double w5[5];
    if (!minnorm_ls(A, b, m, 5, w5)) return HELM27_ENUMERIC;
    for (int k = 0; k < 5; ++k) w5[k] += w0[k];
    helm27_table* t = new (std::nothrow) helm27_table;
    if (!t) return HELM27_ENOMEM;
    t->g_min = g_list[0];
    t->dg = 1.0;
    t->n_g = 1;
    t->w7.resize(7);
    complete_weights(w5, t->w7.data());
    *out = t;
    return HELM27_OK;
}
