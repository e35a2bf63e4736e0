// Householder QR for the orthogonalisation of cluster bases.
#include "linalg.hpp"

namespace h2b {

void householder_qr(int m, int n, const double *A, std::vector<double> &Q, std::vector<double> &R)
{
    const int r = std::min(m, n);
    std::vector<double> a(A, A + (size_t)m * n);
    std::vector<double> V((size_t)r * m, 0.0), beta(r, 0.0);
    for (int j = 0; j < r; ++j) {
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += a[(size_t)i * n + j] * a[(size_t)i * n + j];
        nrm = std::sqrt(nrm);
        double *v = &V[(size_t)j * m];
        if (nrm == 0.0) continue;
        const double ajj = a[(size_t)j * n + j];
        const double alpha = (ajj >= 0.0) ? -nrm : nrm;
        for (int i = j; i < m; ++i) v[i] = a[(size_t)i * n + j];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        beta[j] = 2.0 / vv;
        for (int c = j; c < n; ++c) {
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * a[(size_t)i * n + c];
            s *= beta[j];
            for (int i = j; i < m; ++i) a[(size_t)i * n + c] -= s * v[i];
        }
    }
    R.assign((size_t)r * n, 0.0);
    for (int i = 0; i < r; ++i)
        for (int c = i; c < n; ++c) R[(size_t)i * n + c] = a[(size_t)i * n + c];
    // Q = H_0 H_1 ... H_{r-1} applied to the first r columns of the identity
    Q.assign((size_t)m * r, 0.0);
    for (int i = 0; i < r; ++i) Q[(size_t)i * r + i] = 1.0;
    for (int j = r - 1; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        const double *v = &V[(size_t)j * m];
        for (int c = 0; c < r; ++c) {
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * Q[(size_t)i * r + c];
            s *= beta[j];
            for (int i = j; i < m; ++i) Q[(size_t)i * r + c] -= s * v[i];
        }
    }
}

}  // namespace h2b
