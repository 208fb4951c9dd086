// Host-side construction of least-misfit gridding tables (FP64).
//
// Ye, Gull, Tan & Nikolic (2019): the normal equations A C(nu) = B(nu)
// (Sec. 2.1, Eqs. 17-19), Levenberg-Marquardt optimisation of the correcting
// function h on N_g + 1 = 33 points with M_g = 16 offsets (App. A), table
// generation (App. E), Newton forward interpolation (App. F) and the optimal
// correction (Eqs. 12-15).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "lmg_internal.h"

namespace lmg {

double delta_low(int W) { return (W % 2) ? -0.5 : 0.0; }
double tap_reference(int W) { return (W % 2) ? 0.5 * (W - 1) : 0.5 * W - 1.0; }

namespace {

constexpr double kPi = 3.14159265358979323846;

// In-place Cholesky factorisation of an n x n SPD matrix (lower triangle).
bool cholesky(std::vector<double>& a, int n) {
    for (int j = 0; j < n; ++j) {
        double d = a[j * n + j];
        for (int k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        a[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = a[i * n + j];
            for (int k = 0; k < j; ++k) s -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / d;
        }
    }
    return true;
}

// Solve L L^T x = b for one right-hand side (b overwritten by x).
void cholesky_solve(const std::vector<double>& l, int n, double* b) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= l[i * n + k] * b[k];
        b[i] = s / l[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= l[k * n + i] * b[k];
        b[i] = s / l[i * n + i];
    }
}

// Gauss-Legendre nodes/weights on [a, b] (Newton iteration on P_n).
void gauss_legendre(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = wt;
        w[n - 1 - i] = wt;
    }
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (b - a) * x[i] + 0.5 * (b + a);
        w[i] *= 0.5 * (b - a);
    }
}

// From W = 12 the normal matrix A of Eq. 19 is too ill-conditioned (cond(A)
// 7e7 at W = 12, 1e11 at W = 16) for the Cholesky solve to keep the kernel's
// accuracy; App. B's least-squares form is solved by QR instead.
constexpr int kQrMinW = 12;

// App. B: C(t - delta) as the least-squares solution over the 2 N_g + 1
// symmetric samples x_s of [-x0, x0] (trapezoid weights w_s): rows sqrt(w_s)
// h_s (cos, sin)(2 pi (t_r - delta) x_s) against (sqrt(w_s), 0); its normal
// equations are exactly Eq. 18. A shift of delta rotates each sample's
// (cos, sin) row pair by the angle 2 pi delta x_s, an orthogonal map, so one
// Householder QR of the delta = 0 matrix serves every offset:
// C = R^{-1} Q^T g(delta), g = sqrt(w_s) (cos, sin)(2 pi delta x_s).
struct KernelQR {
    int W = 0, m = 0;
    std::vector<double> a;        // m x W, column-major; Householder vectors from the diagonal down
    std::vector<double> beta, rdiag;
    std::vector<double> xs, sw;   // samples and square roots of their weights

    bool factor(int W_, double x0, const double* h) {
        W = W_;
        const int ns = 2 * kNg + 1;
        m = 2 * ns;
        xs.resize(ns);
        sw.resize(ns);
        std::vector<double> hs(ns);
        for (int s = 0; s < ns; ++s) {
            const int i = s - kNg;                         // -N_g .. N_g
            const int ai = i < 0 ? -i : i;
            xs[s] = i * (x0 / kNg);
            sw[s] = std::sqrt((ai == kNg ? 0.5 : 1.0) * (x0 / kNg));
            hs[s] = h[ai];
        }
        const double ref = tap_reference(W);
        a.assign(static_cast<size_t>(m) * W, 0.0);
        for (int r = 0; r < W; ++r)
            for (int s = 0; s < ns; ++s) {
                const double ph = 2 * kPi * (r - ref) * xs[s];
                a[static_cast<size_t>(r) * m + s] = sw[s] * hs[s] * std::cos(ph);
                a[static_cast<size_t>(r) * m + ns + s] = sw[s] * hs[s] * std::sin(ph);
            }
        beta.assign(W, 0.0);
        rdiag.assign(W, 0.0);
        for (int k = 0; k < W; ++k) {
            double* v = &a[static_cast<size_t>(k) * m];
            double nrm = 0.0;
            for (int i = k; i < m; ++i) nrm += v[i] * v[i];
            nrm = std::sqrt(nrm);
            if (!(nrm > 0.0)) return false;
            const double alpha = v[k] > 0 ? -nrm : nrm;    // R_kk; v = x - alpha e_k avoids cancellation
            v[k] -= alpha;
            double vv = 0.0;
            for (int i = k; i < m; ++i) vv += v[i] * v[i];
            beta[k] = 2.0 / vv;
            rdiag[k] = alpha;
            for (int j = k + 1; j < W; ++j) {
                double* col = &a[static_cast<size_t>(j) * m];
                double sdot = 0.0;
                for (int i = k; i < m; ++i) sdot += v[i] * col[i];
                sdot *= beta[k];
                for (int i = k; i < m; ++i) col[i] -= sdot * v[i];
            }
        }
        return true;
    }

    // c[0..W) = C(t_j - delta).
    void solve(double delta, double* c) const {
        const int ns = m / 2;
        std::vector<double> g(m);
        for (int s = 0; s < ns; ++s) {
            const double b = 2 * kPi * delta * xs[s];
            g[s] = sw[s] * std::cos(b);
            g[ns + s] = sw[s] * std::sin(b);
        }
        for (int k = 0; k < W; ++k) {                      // g <- Q^T g
            const double* v = &a[static_cast<size_t>(k) * m];
            double sdot = 0.0;
            for (int i = k; i < m; ++i) sdot += v[i] * g[i];
            sdot *= beta[k];
            for (int i = k; i < m; ++i) g[i] -= sdot * v[i];
        }
        for (int i = W - 1; i >= 0; --i) {                 // R c = (Q^T g)[0..W)
            double sum = g[i];
            for (int j = i + 1; j < W; ++j) sum -= a[static_cast<size_t>(j) * m + i] * c[j];
            c[i] = sum / rdiag[i];
        }
    }
};

// The optimisation problem for one (W, x0): trigonometric tables that do not
// depend on h are built once.
struct Problem {
    int W;
    double x0;
    std::vector<double> x, tau;           // coarse x grid on [0, x0] and trapezoid weights
    std::vector<double> nu;               // M_g offsets in (0, 1/2)
    std::vector<double> cos_diff;         // [(r' - r) + W - 1][i]
    std::vector<double> cos_b;            // [j][m][i] cos(2 pi (t_j - nu_m) x_i)
    std::vector<double> sin_b;            // [j][m][i]

    Problem(int W_, double x0_) : W(W_), x0(x0_) {
        x.resize(kNg + 1);
        tau.resize(kNg + 1);
        for (int i = 0; i <= kNg; ++i) {
            x[i] = i * (x0 / kNg);
            tau[i] = x0 / kNg;
        }
        tau[0] *= 0.5;
        tau[kNg] *= 0.5;
        nu.resize(kMg);
        for (int m = 0; m < kMg; ++m) nu[m] = (m + 0.5) / (2.0 * kMg);
        cos_diff.resize((2 * W - 1) * (kNg + 1));
        for (int d = -(W - 1); d <= W - 1; ++d)
            for (int i = 0; i <= kNg; ++i) cos_diff[(d + W - 1) * (kNg + 1) + i] = std::cos(2 * kPi * d * x[i]);
        cos_b.resize(W * kMg * (kNg + 1));
        sin_b.resize(W * kMg * (kNg + 1));
        const double ref = tap_reference(W);
        for (int j = 0; j < W; ++j)
            for (int m = 0; m < kMg; ++m)
                for (int i = 0; i <= kNg; ++i) {
                    double ph = 2 * kPi * ((j - ref) - nu[m]) * x[i];
                    cos_b[(j * kMg + m) * (kNg + 1) + i] = std::cos(ph);
                    sin_b[(j * kMg + m) * (kNg + 1) + i] = std::sin(ph);
                }
    }

    // A_{r'r} = 2 sum_i tau_i h_i^2 cos(2 pi (r' - r) x_i)   (Eq. 19)
    void normal_matrix(const double* h, std::vector<double>& A) const {
        A.assign(W * W, 0.0);
        std::vector<double> wd(2 * W - 1, 0.0);
        for (int d = 0; d < 2 * W - 1; ++d) {
            double s = 0.0;
            for (int i = 0; i <= kNg; ++i) s += tau[i] * h[i] * h[i] * cos_diff[d * (kNg + 1) + i];
            wd[d] = 2.0 * s;
        }
        for (int a = 0; a < W; ++a)
            for (int b = 0; b < W; ++b) A[a * W + b] = wd[a - b + W - 1];
    }

    // Residuals rho_{i,m} = sqrt(tau_i / (x0 M_g)) (1 - h_i S(nu_m, x_i)), (Re, Im), App. A.
    bool residuals(const double* h, double* r) const {
        std::vector<double> A;
        KernelQR qr;
        if (W >= kQrMinW) {
            if (!qr.factor(W, x0, h)) return false;
        } else {
            normal_matrix(h, A);
            if (!cholesky(A, W)) return false;
        }
        std::vector<double> c(W);
        for (int m = 0; m < kMg; ++m) {
            if (W >= kQrMinW) {
                qr.solve(nu[m], c.data());
            } else {
                for (int j = 0; j < W; ++j) {           // B_{r'}(nu) = 2 sum tau h cos(...)  (Eq. 18)
                    double s = 0.0;
                    const double* cb = &cos_b[(j * kMg + m) * (kNg + 1)];
                    for (int i = 0; i <= kNg; ++i) s += tau[i] * h[i] * cb[i];
                    c[j] = 2.0 * s;
                }
                cholesky_solve(A, W, c.data());
            }
            for (int i = 0; i <= kNg; ++i) {
                double sr = 0.0, si = 0.0;
                for (int j = 0; j < W; ++j) {
                    sr += c[j] * cos_b[(j * kMg + m) * (kNg + 1) + i];
                    si += c[j] * sin_b[(j * kMg + m) * (kNg + 1) + i];
                }
                const double wgt = std::sqrt(tau[i] / (x0 * kMg));
                r[(m * (kNg + 1) + i)] = wgt * (1.0 - h[i] * sr);
                r[kMg * (kNg + 1) + (m * (kNg + 1) + i)] = wgt * (-h[i] * si);
            }
        }
        return true;
    }
    int nres() const { return 2 * kMg * (kNg + 1); }
};

double sumsq(const std::vector<double>& r) {
    double s = 0.0;
    for (double v : r) s += v * v;
    return s;
}

// Levenberg-Marquardt over h_1 .. h_Ng with h_0 = 1 fixed (E is invariant
// under h -> a h). Central-difference Jacobian, multiplicative damping on
// diag(J^T J). Returns false if no finite starting point.
bool levenberg_marquardt(const Problem& P, std::vector<double>& h, double* E_out) {
    const int n = kNg, m = P.nres();
    std::vector<double> r(m), rt(m), rp(m), rm(m), J(static_cast<size_t>(m) * n);
    if (!P.residuals(h.data(), r.data())) return false;
    double E = sumsq(r);
    double lambda = 1e-3;
    int stall = 0;
    std::vector<double> H(n * n), g(n), M(n * n), step(n), ht(kNg + 1);
    for (int iter = 0; iter < 2000 && stall < 4; ++iter) {
        for (int k = 0; k < n; ++k) {
            const double hk = h[k + 1];
            const double d = 1e-6 * std::max(1.0, std::fabs(hk));
            h[k + 1] = hk + d;
            P.residuals(h.data(), rp.data());
            h[k + 1] = hk - d;
            P.residuals(h.data(), rm.data());
            h[k + 1] = hk;
            for (int i = 0; i < m; ++i) J[static_cast<size_t>(i) * n + k] = (rp[i] - rm[i]) / (2 * d);
        }
        for (int a = 0; a < n; ++a) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += J[static_cast<size_t>(i) * n + a] * r[i];
            g[a] = s;
            for (int b = 0; b <= a; ++b) {
                double t = 0.0;
                for (int i = 0; i < m; ++i) t += J[static_cast<size_t>(i) * n + a] * J[static_cast<size_t>(i) * n + b];
                H[a * n + b] = H[b * n + a] = t;
            }
        }
        bool accepted = false;
        for (int tries = 0; tries < 30; ++tries) {
            M = H;
            for (int a = 0; a < n; ++a) M[a * n + a] += lambda * std::max(H[a * n + a], 1e-300);
            if (!cholesky(M, n)) { lambda *= 10.0; continue; }
            for (int a = 0; a < n; ++a) step[a] = -g[a];
            cholesky_solve(M, n, step.data());
            ht = h;
            for (int a = 0; a < n; ++a) ht[a + 1] += step[a];
            if (P.residuals(ht.data(), rt.data())) {
                const double Et = sumsq(rt);
                if (std::isfinite(Et) && Et < E) {
                    const double rel = (E - Et) / E;
                    double sn = 0.0, hn = 0.0;
                    for (int a = 0; a < n; ++a) { sn += step[a] * step[a]; hn += ht[a + 1] * ht[a + 1]; }
                    h = ht;
                    r = rt;
                    E = Et;
                    lambda = std::max(lambda * 0.1, 1e-15);
                    accepted = true;
                    stall = (rel < 1e-9 || std::sqrt(sn) < 1e-13 * std::sqrt(hn)) ? stall + 1 : 0;
                    break;
                }
            }
            lambda *= 10.0;
            if (lambda > 1e20) break;
        }
        if (!accepted) break;
    }
    *E_out = E;
    return true;
}

// C(t_j - delta_k) = [A^{-1} B(delta_k)]_j for a given h (Eq. 18).
bool exact_kernel(int W, double x0, const std::vector<double>& h, const double* delta, int n, double* out) {
    if (W >= kQrMinW) {
        KernelQR qr;
        if (!qr.factor(W, x0, h.data())) return false;
        for (int k = 0; k < n; ++k) qr.solve(delta[k], out + static_cast<size_t>(k) * W);
        return true;
    }
    Problem P(W, x0);
    std::vector<double> A;
    P.normal_matrix(h.data(), A);
    if (!cholesky(A, W)) return false;
    const double ref = tap_reference(W);
    for (int k = 0; k < n; ++k) {
        double* c = out + static_cast<size_t>(k) * W;
        for (int j = 0; j < W; ++j) {
            double s = 0.0;
            for (int i = 0; i <= kNg; ++i) s += P.tau[i] * h[i] * std::cos(2 * kPi * ((j - ref) - delta[k]) * P.x[i]);
            c[j] = 2.0 * s;
        }
        cholesky_solve(A, W, c);
    }
    return true;
}

// Expansion of the exact kernel over the h samples (Eq. 18 with Eq. 19's
// quadrature): B_r(delta) = 2 sum_i tau_i h_i cos(2 pi (t_r - delta) x_i)
// splits by the angle-difference identity into cos(2 pi t_r x_i) cos(2 pi
// delta x_i) + sin(2 pi t_r x_i) sin(2 pi delta x_i), so C = A^{-1} B is
// sum_i P_i cos(i theta) + Q_i sin(i theta) with theta = 2 pi delta x0 / N_g,
// P_i = A^{-1} (2 tau_i h_i cos(2 pi t x_i)), Q_i = A^{-1} (2 tau_i h_i sin(2 pi t x_i)).
bool direct_coefficients(int W, double x0, const std::vector<double>& h, std::vector<double>& pq) {
    Problem P(W, x0);
    std::vector<double> A;
    P.normal_matrix(h.data(), A);
    if (!cholesky(A, W)) return false;
    const double ref = tap_reference(W);
    const int ni = kNg + 1;
    pq.assign(2 * static_cast<size_t>(W) * ni + 1, 0.0);
    std::vector<double> c(W), sn(W);
    for (int i = 0; i < ni; ++i) {
        for (int r = 0; r < W; ++r) {
            const double ph = 2 * kPi * (r - ref) * P.x[i];
            c[r] = 2.0 * P.tau[i] * h[i] * std::cos(ph);
            sn[r] = 2.0 * P.tau[i] * h[i] * std::sin(ph);
        }
        cholesky_solve(A, W, c.data());
        cholesky_solve(A, W, sn.data());
        for (int j = 0; j < W; ++j) {
            pq[static_cast<size_t>(j) * ni + i] = c[j];
            pq[static_cast<size_t>(W + j) * ni + i] = sn[j];
        }
    }
    pq[2 * static_cast<size_t>(W) * ni] = 2 * kPi * x0 / kNg;
    return true;
}

bool valid_params(int W, double x0, int table_size, int degree) {
    return W >= 1 && W <= kMaxW && x0 > 0.0 && x0 <= 0.5 && table_size >= W && degree >= 0 && degree <= 3 &&
           (table_size / W) >= 2;
}

// Newton forward-difference polynomial of each table interval, re-expanded
// in powers of t (App. F).
void build_coefficients(lmg_table* t) {
    const int W = t->W, Ms = t->Ms, d = t->degree, ncol = Ms + 1 + d;
    t->coef64.assign(static_cast<size_t>(Ms + 1) * W * 4, 0.0);
    for (int k = 0; k <= Ms; ++k)
        for (int j = 0; j < W; ++j) {
            const double* f = &t->nodes[static_cast<size_t>(j) * ncol + k];
            double c0 = f[0], c1 = 0, c2 = 0, c3 = 0;
            if (d >= 1) {
                const double d1 = f[1] - f[0];
                c1 = d1;
                if (d >= 2) {
                    const double d2 = f[2] - 2 * f[1] + f[0];
                    c1 -= 0.5 * d2;
                    c2 = 0.5 * d2;
                    if (d >= 3) {
                        const double d3 = f[3] - 3 * f[2] + 3 * f[1] - f[0];
                        c1 += d3 / 3.0;
                        c2 -= 0.5 * d3;
                        c3 = d3 / 6.0;
                    }
                }
            }
            double* o = &t->coef64[(static_cast<size_t>(k) * W + j) * 4];
            o[0] = c0; o[1] = c1; o[2] = c2; o[3] = c3;
        }
    t->coef32.resize(t->coef64.size());
    for (size_t i = 0; i < t->coef64.size(); ++i) t->coef32[i] = static_cast<float>(t->coef64[i]);
}

lmg_status finish_table(lmg_table* t, int table_size) {
    t->Ms = table_size / t->W;
    const int ncol = t->Ms + 1 + t->degree;
    std::vector<double> deltas(ncol);
    for (int i = 0; i < ncol; ++i) deltas[i] = delta_low(t->W) + static_cast<double>(i) / t->Ms;
    std::vector<double> kv(static_cast<size_t>(ncol) * t->W);
    if (!exact_kernel(t->W, t->x0, t->h, deltas.data(), ncol, kv.data())) return LMG_EINVAL;
    t->nodes.assign(static_cast<size_t>(t->W) * ncol, 0.0);
    for (int i = 0; i < ncol; ++i)
        for (int j = 0; j < t->W; ++j) t->nodes[static_cast<size_t>(j) * ncol + i] = kv[static_cast<size_t>(i) * t->W + j];
    build_coefficients(t);
    return LMG_OK;
}

double coarse_misfit(int W, double x0, const std::vector<double>& h) {
    Problem P(W, x0);
    std::vector<double> r(P.nres());
    std::vector<double> hs(h);
    for (double& v : hs) v /= h[0];
    if (!P.residuals(hs.data(), r.data())) return NAN;
    return sumsq(r);
}

// Optimal h for (W, x0) through App. A's chain of initial guesses.
bool optimal_h(int W, double x0, std::vector<double>& h, double* E) {
    std::vector<std::vector<double>> hs(W + 1);
    for (int w = (W <= 4 ? W : 3); w <= W; ++w) {
        std::vector<double> init(kNg + 1, 1.0);
        if (w > 4)
            for (int i = 0; i <= kNg; ++i) init[i] = hs[w - 1][i] * hs[w - 1][i] / hs[w - 2][i];
        Problem P(w, x0);
        double Ew = 0;
        if (!levenberg_marquardt(P, init, &Ew)) return false;
        hs[w] = init;
        if (w == W) *E = Ew;
    }
    h = hs[W];
    return true;
}

// S(delta, x) = sum_j C_j(delta) exp(i 2 pi (t_j - delta) x) accumulated into
// c(x) = int Re S, D(x) = int |S|^2 and, given h(x), l(x) = int |1 - h S|^2.
void nu_integrals(int W, const std::vector<double>& qd, const std::vector<double>& qw, const std::vector<double>& kv,
                  double x, double hx, bool use_h, double* c, double* D, double* ell) {
    const double ref = tap_reference(W);
    double cs = 0, ds = 0, es = 0;
    for (size_t q = 0; q < qd.size(); ++q) {
        double sr = 0, si = 0;
        for (int j = 0; j < W; ++j) {
            const double ph = 2 * kPi * ((j - ref) - qd[q]) * x;
            sr += kv[q * W + j] * std::cos(ph);
            si += kv[q * W + j] * std::sin(ph);
        }
        cs += qw[q] * sr;
        ds += qw[q] * (sr * sr + si * si);
        if (use_h) {
            const double er = 1.0 - hx * sr, ei = -hx * si;
            es += qw[q] * (er * er + ei * ei);
        }
    }
    *c = cs;
    *D = ds;
    if (ell) *ell = es;
}

// Host evaluation of the tabulated kernel (same rule as the device).
void table_weights(const lmg_table* t, double delta, double* out) {
    const double p = (delta - delta_low(t->W)) * t->Ms;
    if (t->degree == 0) {
        int k = static_cast<int>(std::floor(p + 0.5));
        k = std::min(std::max(k, 0), t->Ms);
        for (int j = 0; j < t->W; ++j) out[j] = t->coef64[(static_cast<size_t>(k) * t->W + j) * 4];
        return;
    }
    int k = static_cast<int>(std::floor(p));
    k = std::min(std::max(k, 0), t->Ms);
    const double s = p - k;
    for (int j = 0; j < t->W; ++j) {
        const double* c = &t->coef64[(static_cast<size_t>(k) * t->W + j) * 4];
        out[j] = c[0] + s * (c[1] + s * (c[2] + s * c[3]));
    }
}

}  // namespace
}  // namespace lmg

using namespace lmg;

extern "C" {

lmg_status lmg_table_create(int W, double x0, int table_size, int degree, lmg_table** out) {
    if (!out || !valid_params(W, x0, table_size, degree)) return LMG_EINVAL;
    std::unique_ptr<lmg_table> t(new (std::nothrow) lmg_table);
    if (!t) return LMG_EINVAL;
    t->W = W;
    t->x0 = x0;
    t->degree = degree;
    if (!optimal_h(W, x0, t->h, &t->E)) return LMG_ENOCONV;
    lmg_status s = finish_table(t.get(), table_size);
    if (s != LMG_OK) return s;
    *out = t.release();
    return LMG_OK;
}

lmg_status lmg_table_create_from_h(int W, double x0, int table_size, int degree, const double* h_coarse,
                                   lmg_table** out) {
    if (!out || !h_coarse || !valid_params(W, x0, table_size, degree)) return LMG_EINVAL;
    std::unique_ptr<lmg_table> t(new (std::nothrow) lmg_table);
    if (!t) return LMG_EINVAL;
    t->W = W;
    t->x0 = x0;
    t->degree = degree;
    t->h.assign(h_coarse, h_coarse + kNg + 1);
    for (double v : t->h)
        if (!std::isfinite(v) || v == 0.0) return LMG_EINVAL;
    t->E = coarse_misfit(W, x0, t->h);
    lmg_status s = finish_table(t.get(), table_size);
    if (s != LMG_OK) return s;
    *out = t.release();
    return LMG_OK;
}

lmg_status lmg_table_create_from_nodes(int W, double x0, int table_size, int degree, const double* h_coarse,
                                       const double* nodes, lmg_table** out) {
    if (!out || !h_coarse || !nodes || !valid_params(W, x0, table_size, degree)) return LMG_EINVAL;
    std::unique_ptr<lmg_table> t(new (std::nothrow) lmg_table);
    if (!t) return LMG_EINVAL;
    t->W = W;
    t->x0 = x0;
    t->degree = degree;
    t->Ms = table_size / W;
    t->h.assign(h_coarse, h_coarse + kNg + 1);
    const size_t nn = static_cast<size_t>(W) * (t->Ms + 1 + degree);
    t->nodes.assign(nodes, nodes + nn);
    for (double v : t->nodes)
        if (!std::isfinite(v)) return LMG_EINVAL;
    t->E = coarse_misfit(W, x0, t->h);
    build_coefficients(t.get());
    *out = t.release();
    return LMG_OK;
}

lmg_status lmg_table_create_direct(const lmg_table* from, lmg_table** out) {
    if (!from || !out) return LMG_EINVAL;
    std::unique_ptr<lmg_table> t(new (std::nothrow) lmg_table);
    if (!t) return LMG_EINVAL;
    t->W = from->W;
    t->x0 = from->x0;
    t->Ms = from->Ms;
    t->degree = from->degree;
    t->E = from->E;
    t->h = from->h;
    t->nodes = from->nodes;
    t->coef32 = from->coef32;
    t->coef64 = from->coef64;
    // The expansion multiplies by A^{-1} (cond(A) eps cancellation): from W = 12 it no longer holds FP64
    // accuracy, and the QR form of App. B has no fixed expansion of this kind.
    if (t->W >= kQrMinW) return LMG_ENOTSUP;
    t->direct = true;
    if (!direct_coefficients(t->W, t->x0, t->h, t->pq)) return LMG_EINVAL;
    *out = t.release();
    return LMG_OK;
}

lmg_status lmg_table_device_bytes(const lmg_table* t, lmg_precision prec, size_t* bytes) {
    if (!t || !bytes || prec < LMG_F32 || prec > LMG_F64) return LMG_EINVAL;
    const size_t b = prec == LMG_F64 ? t->coef64.size() * sizeof(double) : t->coef32.size() * sizeof(float);
    *bytes = (t->direct || b <= kMaxLdsTableBytes) ? 0 : b;
    return LMG_OK;
}

lmg_status lmg_table_attach_device(lmg_table* t, lmg_precision prec, void* device, size_t bytes, void* stream) {
    size_t need = 0;
    const lmg_status st = lmg_table_device_bytes(t, prec, &need);
    if (st != LMG_OK) return st;
    if (need == 0) return LMG_OK;                      // the kernels stage this table in LDS
    if (!device || bytes < need) return LMG_EWORKSPACE;
    const int i = prec == LMG_F64 ? 1 : 0;
    const void* src = i ? static_cast<const void*>(t->coef64.data()) : static_cast<const void*>(t->coef32.data());
    if (hipMemcpyAsync(device, src, need, hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)) != hipSuccess)
        return LMG_EHIP;
    // (pageable host memory: the copy has left the host buffer when hipMemcpyAsync returns)
    t->dev_coef[i] = device;
    t->dev_bytes[i] = need;
    return LMG_OK;
}

lmg_status lmg_table_is_direct(const lmg_table* t, int* direct) {
    if (!t || !direct) return LMG_EINVAL;
    *direct = t->direct ? 1 : 0;
    return LMG_OK;
}

lmg_status lmg_table_info(const lmg_table* t, int* W, double* x0, int* Ms, int* degree, double* E) {
    if (!t) return LMG_EINVAL;
    if (W) *W = t->W;
    if (x0) *x0 = t->x0;
    if (Ms) *Ms = t->Ms;
    if (degree) *degree = t->degree;
    if (E) *E = t->E;
    return LMG_OK;
}

lmg_status lmg_table_export(const lmg_table* t, double* h_coarse, double* nodes) {
    if (!t) return LMG_EINVAL;
    if (h_coarse) std::memcpy(h_coarse, t->h.data(), sizeof(double) * t->h.size());
    if (nodes) std::memcpy(nodes, t->nodes.data(), sizeof(double) * t->nodes.size());
    return LMG_OK;
}

lmg_status lmg_table_kernel(const lmg_table* t, int n, const double* delta, double* out) {
    if (!t || n < 0 || (n > 0 && (!delta || !out))) return LMG_EINVAL;
    return exact_kernel(t->W, t->x0, t->h, delta, n, out) ? LMG_OK : LMG_EINVAL;
}

lmg_status lmg_correction(const lmg_table* t, int N, double* h_pix) {
    if (!t || !h_pix || N < 2 || (N & (N - 1))) return LMG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(t->cache_mu);
        auto it = t->hpix_cache.find(N);
        if (it != t->hpix_cache.end()) {
            std::memcpy(h_pix, it->second.data(), sizeof(double) * N);
            return LMG_OK;
        }
    }
    std::vector<double> qd, qw;
    gauss_legendre(64, delta_low(t->W), delta_low(t->W) + 1.0, qd, qw);
    std::vector<double> kv(qd.size() * t->W);
    if (!exact_kernel(t->W, t->x0, t->h, qd.data(), static_cast<int>(qd.size()), kv.data())) return LMG_EINVAL;
    // h is even: evaluate p = 0 .. N/2 and mirror.
    for (int p = 0; p <= N / 2; ++p) {
        double c, D;
        nu_integrals(t->W, qd, qw, kv, static_cast<double>(p) / N, 0.0, false, &c, &D, nullptr);
        const double hv = c / D;
        if (p < N / 2) h_pix[N / 2 + p] = hv;
        h_pix[N / 2 - p] = hv;
    }
    std::lock_guard<std::mutex> lk(t->cache_mu);
    t->hpix_cache[N].assign(h_pix, h_pix + N);
    return LMG_OK;
}

lmg_status lmg_map_error(const lmg_table* t, int n, const double* x, double* ell_exact, double* ell_table) {
    if (!t || n < 0 || (n > 0 && !x)) return LMG_EINVAL;
    const double lo = delta_low(t->W);
    std::vector<double> qd, qw;
    gauss_legendre(64, lo, lo + 1.0, qd, qw);
    std::vector<double> kv(qd.size() * t->W);
    if (!exact_kernel(t->W, t->x0, t->h, qd.data(), static_cast<int>(qd.size()), kv.data())) return LMG_EINVAL;
    // Composite rule for the piecewise-polynomial table kernel: 8 GL points per table interval.
    std::vector<double> td, tw, gx, gw;
    gauss_legendre(8, 0.0, 1.0 / t->Ms, gx, gw);
    for (int k = 0; k < t->Ms; ++k)
        for (int q = 0; q < 8; ++q) {
            td.push_back(lo + static_cast<double>(k) / t->Ms + gx[q]);
            tw.push_back(gw[q]);
        }
    std::vector<double> tv(td.size() * t->W);
    if (t->direct) {                      // no table: the kernels evaluate the exact kernel
        if (!exact_kernel(t->W, t->x0, t->h, td.data(), static_cast<int>(td.size()), tv.data())) return LMG_EINVAL;
    } else {
        for (size_t q = 0; q < td.size(); ++q) table_weights(t, td[q], &tv[q * t->W]);
    }
    for (int i = 0; i < n; ++i) {
        double c, D, e;
        nu_integrals(t->W, qd, qw, kv, x[i], 0.0, false, &c, &D, nullptr);
        const double hx = c / D;
        if (ell_exact) {
            nu_integrals(t->W, qd, qw, kv, x[i], hx, true, &c, &D, &e);
            ell_exact[i] = e;
        }
        if (ell_table) {
            nu_integrals(t->W, td, tw, tv, x[i], hx, true, &c, &D, &e);
            ell_table[i] = e;
        }
    }
    return LMG_OK;
}

void lmg_table_destroy(lmg_table* t) { delete t; }

const char* lmg_status_string(lmg_status s) {
    switch (s) {
        case LMG_OK: return "ok";
        case LMG_EINVAL: return "invalid argument";
        case LMG_EWORKSPACE: return "workspace missing or too small";
        case LMG_EHIP: return "HIP runtime error";
        case LMG_EDATA: return "non-finite uv coordinates were dropped";
        case LMG_ENOTSUP: return "valid request the library does not support";
        case LMG_ENOCONV: return "table optimisation did not converge";
    }
    return "unknown status";
}

}  // extern "C"

lmg_table::~lmg_table() {
    for (auto& kv : pinned)
        if (kv.second.host) (void)hipHostFree(kv.second.host);
}
