// Ritz step of Appendix A on the host: eigenpairs of the small m x m upper
// Hessenberg matrix H_m (m <= a few hundred) produced by the Arnoldi process.
//
// Eigenvalues: implicitly shifted Francis double-shift QR iteration on the
// active diagonal window (Golub & Van Loan, Sect. 7.5), deflating when a
// subdiagonal entry becomes negligible, reading 1x1 and 2x2 blocks off at the
// bottom.  Eigenvectors: inverse iteration on H - theta I with a Hessenberg LU
// (partial pivoting) in complex arithmetic.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "mm_internal.h"

namespace mm {
namespace {

using cd = std::complex<double>;

struct Mat {
    int n;
    std::vector<double> a;  // row-major
    double &operator()(int i, int j) { return a[(size_t)i * n + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

// Householder vector v (v[0] = 1) and beta with (I - beta v v^T) x = alpha e1.
void house(const double *x, int len, double *v, double &beta) {
    double sigma = 0;
    for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
    v[0] = 1;
    for (int i = 1; i < len; ++i) v[i] = x[i];
    if (sigma == 0) {
        beta = 0;
        return;
    }
    const double mu = std::sqrt(x[0] * x[0] + sigma);
    const double v0 = x[0] <= 0 ? x[0] - mu : -sigma / (x[0] + mu);
    beta = 2 * v0 * v0 / (sigma + v0 * v0);
    for (int i = 1; i < len; ++i) v[i] /= v0;
}

// Apply (I - beta v v^T) from the left to rows r0..r0+len-1, columns c0..c1,
// and from the right to columns r0..r0+len-1, rows q0..q1.
void reflect(Mat &H, int r0, int len, const double *v, double beta, int c0, int c1, int q0,
             int q1) {
    if (beta == 0) return;
    for (int c = c0; c <= c1; ++c) {
        double s = 0;
        for (int i = 0; i < len; ++i) s += v[i] * H(r0 + i, c);
        s *= beta;
        for (int i = 0; i < len; ++i) H(r0 + i, c) -= s * v[i];
    }
    for (int q = q0; q <= q1; ++q) {
        double s = 0;
        for (int i = 0; i < len; ++i) s += H(q, r0 + i) * v[i];
        s *= beta;
        for (int i = 0; i < len; ++i) H(q, r0 + i) -= s * v[i];
    }
}

void eig2(double a, double b, double c, double d, cd &e1, cd &e2) {
    const double p = 0.5 * (a - d);
    const double disc = p * p + b * c;
    const double mid = 0.5 * (a + d);
    if (disc >= 0) {
        const double sq = std::sqrt(disc);
        // avoid cancellation: the larger-magnitude root mid +- sq takes the
        // sign of mid, the other one follows from the determinant
        const double r1 = mid + (mid >= 0 ? sq : -sq);
        const double prod = a * d - b * c;
        const double r2 = r1 != 0 ? prod / r1 : mid - (mid >= 0 ? sq : -sq);
        e1 = cd(r1, 0);
        e2 = cd(r2, 0);
    } else {
        const double sq = std::sqrt(-disc);
        e1 = cd(mid, -sq);
        e2 = cd(mid, sq);
    }
}

std::vector<cd> hqr_eigenvalues(Mat H) {
    const int n = H.n;
    std::vector<cd> ev;
    ev.reserve(n);
    const double eps = 2.220446049250313e-16;
    double hnorm = 0;
    for (double x : H.a) hnorm = std::max(hnorm, std::fabs(x));
    int u = n - 1;
    int iter = 0, total = 0;
    while (u >= 0) {
        int l = u;
        while (l > 0) {
            double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (s == 0) s = hnorm;
            if (std::fabs(H(l, l - 1)) <= eps * s) {
                H(l, l - 1) = 0;
                break;
            }
            --l;
        }
        if (l == u) {
            ev.push_back(cd(H(u, u), 0));
            --u;
            iter = 0;
            continue;
        }
        if (l == u - 1) {
            cd e1, e2;
            eig2(H(u - 1, u - 1), H(u - 1, u), H(u, u - 1), H(u, u), e1, e2);
            ev.push_back(e1);
            ev.push_back(e2);
            u -= 2;
            iter = 0;
            continue;
        }
        MM_CHECK(total < 30 * std::max(10, n) * 4, MM_E_DEVICE, "Hessenberg QR did not converge");
        ++iter;
        ++total;
        double s, t;
        if (iter % 10 == 0) {
            // exceptional shifts, centred on a diagonal entry of the window:
            // the eigenvalues of [[a, -0.4375 w], [w, a]] with a = h + 0.75 w,
            // w the size of two neighbouring subdiagonals -- alternately at the
            // bottom (h = H(u,u)) and at the top (h = H(l,l)) of the window.
            // They break the cycles the standard shifts can fall into on tight
            // clusters of eigenvalues.
            const bool top = (iter / 10) % 2 == 0;
            const double w = top ? std::fabs(H(l + 1, l)) + std::fabs(H(l + 2, l + 1))
                                 : std::fabs(H(u, u - 1)) + std::fabs(H(u - 1, u - 2));
            const double a = (top ? H(l, l) : H(u, u)) + 0.75 * w;
            s = 2.0 * a;
            t = a * a + 0.4375 * w * w;
        } else {
            s = H(u - 1, u - 1) + H(u, u);
            t = H(u - 1, u - 1) * H(u, u) - H(u - 1, u) * H(u, u - 1);
        }
        double x = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
        double y = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
        double z = H(l + 1, l) * H(l + 2, l + 1);
        double v[3], beta;
        for (int k = l; k <= u - 2; ++k) {
            const double xv[3] = {x, y, z};
            house(xv, 3, v, beta);
            const int c0 = std::max(l, k - 1);
            const int q1 = std::min(k + 3, u);
            reflect(H, k, 3, v, beta, c0, u, l, q1);
            x = H(k + 1, k);
            y = H(k + 2, k);
            if (k < u - 2) z = H(k + 3, k);
        }
        const double xv2[2] = {x, y};
        house(xv2, 2, v, beta);
        reflect(H, u - 1, 2, v, beta, u - 2, u, l, u);
    }
    return ev;
}

// Solve (H - theta I) y = b for upper Hessenberg H by LU with partial pivoting
// between adjacent rows (Hessenberg structure keeps it O(m^2)).
void hess_solve(const Mat &H, cd theta, std::vector<cd> &b) {
    const int n = H.n;
    std::vector<cd> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            A[(size_t)i * n + j] = (j >= i - 1) ? cd(H(i, j), 0) - (i == j ? theta : cd(0)) : cd(0);
    for (int k = 0; k < n - 1; ++k) {
        cd &piv = A[(size_t)k * n + k];
        cd &sub = A[(size_t)(k + 1) * n + k];
        if (std::abs(sub) > std::abs(piv)) {
            for (int j = k; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)(k + 1) * n + j]);
            std::swap(b[k], b[k + 1]);
        }
        cd p = A[(size_t)k * n + k];
        if (p == cd(0)) p = A[(size_t)k * n + k] = cd(1e-300, 0);
        const cd f = A[(size_t)(k + 1) * n + k] / p;
        for (int j = k; j < n; ++j) A[(size_t)(k + 1) * n + j] -= f * A[(size_t)k * n + j];
        b[k + 1] -= f * b[k];
    }
    for (int i = n - 1; i >= 0; --i) {
        cd s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[(size_t)i * n + j] * b[j];
        cd p = A[(size_t)i * n + i];
        if (p == cd(0)) p = cd(1e-300, 0);
        b[i] = s / p;
    }
}

}  // namespace

// Eigen-decomposition of a small symmetric matrix (cyclic Jacobi rotations):
// A (n x n, row-major) is destroyed; w = eigenvalues, U column j = vector j.
void sym_eig_jacobi(int n, std::vector<double> &A, std::vector<double> &w,
                           std::vector<double> &U) {
    U.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-30 * tot) break;
        for (int pq = 0; pq < n * n; ++pq) {
            const int pi = pq / n, qi = pq % n;
            if (qi <= pi) continue;
            const double apq = A[(size_t)pi * n + qi];
            if (apq == 0.0) continue;
            const double app = A[(size_t)pi * n + pi], aqq = A[(size_t)qi * n + qi];
            const double th = 0.5 * (aqq - app) / apq;
            const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
            const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
            for (int r = 0; r < n; ++r) {  // A <- A J (columns pi, qi)
                const double x = A[(size_t)r * n + pi], y = A[(size_t)r * n + qi];
                A[(size_t)r * n + pi] = c * x - sn * y;
                A[(size_t)r * n + qi] = sn * x + c * y;
            }
            for (int r = 0; r < n; ++r) {  // A <- J^T A (rows pi, qi)
                const double x = A[(size_t)pi * n + r], y = A[(size_t)qi * n + r];
                A[(size_t)pi * n + r] = c * x - sn * y;
                A[(size_t)qi * n + r] = sn * x + c * y;
            }
            for (int r = 0; r < n; ++r) {  // U <- U J
                const double x = U[(size_t)r * n + pi], y = U[(size_t)r * n + qi];
                U[(size_t)r * n + pi] = c * x - sn * y;
                U[(size_t)r * n + qi] = sn * x + c * y;
            }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

void hessenberg_eig(int m, const double *Hcm, double *wr, double *wi, double *vr, double *vi) {
    Mat H{m, std::vector<double>((size_t)m * m)};
    double hnorm = 0;
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            H(i, j) = (i <= j + 1) ? Hcm[(size_t)j * m + i] : 0.0;
            hnorm = std::max(hnorm, std::fabs(H(i, j)));
        }
    std::vector<cd> ev;
    try {
        ev = hqr_eigenvalues(H);
    } catch (const Error &) {
        // QR can stall on tight clusters of a symmetric matrix (a Lanczos
        // tridiagonal whose converged Ritz values repeat): there the Jacobi
        // rotations give eigenvalues and orthonormal eigenvectors directly
        double asym = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < i; ++j) asym = std::max(asym, std::fabs(H(i, j) - H(j, i)));
        if (!(asym <= 1e-12 * std::max(hnorm, 1e-300))) throw;
        std::vector<double> A(H.a), w, U;
        sym_eig_jacobi(m, A, w, U);
        std::vector<int> order(m);
        for (int i = 0; i < m; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int p, int q) { return w[p] < w[q]; });
        for (int i = 0; i < m; ++i) {
            wr[i] = w[order[i]];
            wi[i] = 0.0;
            for (int q = 0; q < m; ++q) {
                vr[(size_t)i * m + q] = U[(size_t)q * m + order[i]];
                vi[(size_t)i * m + q] = 0.0;
            }
        }
        return;
    }
    std::sort(ev.begin(), ev.end(), [](const cd &a, const cd &b) {
        return a.real() != b.real() ? a.real() < b.real() : a.imag() < b.imag();
    });
    const double eps = 2.220446049250313e-16;
    for (int i = 0; i < m; ++i) {
        wr[i] = ev[i].real();
        wi[i] = ev[i].imag();
        // inverse iteration from a fixed start vector
        const cd shift = ev[i] + cd(eps * std::max(hnorm, 1e-300) * 16, 0);
        std::vector<cd> y(m, cd(1.0, 0.0));
        for (int it = 0; it < 3; ++it) {
            hess_solve(H, shift, y);
            double nrm = 0;
            for (auto &c : y) nrm += std::norm(c);
            nrm = std::sqrt(nrm);
            for (auto &c : y) c /= nrm;
        }
        // fix the phase: largest component real and positive
        int imax = 0;
        for (int q = 1; q < m; ++q)
            if (std::abs(y[q]) > std::abs(y[imax])) imax = q;
        const cd ph = std::conj(y[imax]) / std::abs(y[imax]);
        for (auto &c : y) c *= ph;
        const bool real = ev[i].imag() == 0.0;
        for (int q = 0; q < m; ++q) {
            vr[(size_t)i * m + q] = y[q].real();
            vi[(size_t)i * m + q] = real ? 0.0 : y[q].imag();
        }
        if (real) {
            double nrm = 0;
            for (int q = 0; q < m; ++q) nrm += vr[(size_t)i * m + q] * vr[(size_t)i * m + q];
            nrm = std::sqrt(nrm);
            for (int q = 0; q < m; ++q) vr[(size_t)i * m + q] /= nrm;
        }
    }
}

}  // namespace mm
