// Small dense linear algebra on the host (row-major, double), used to set up
// the recompressed cluster bases, and a simple parallel loop.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace h2b {

// Runs f(i) for i in [0, n) on up to hardware_concurrency() threads (at most
// OMP_NUM_THREADS when that is set, and 64).  An exception thrown by f stops
// the remaining work and is rethrown on the calling thread.
template <class F> void parallel_for(int64_t n, F f)
{
    if (n <= 0) return;
    int nt = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 64);
    if (const char *e = std::getenv("OMP_NUM_THREADS")) {
        const int lim = std::atoi(e);
        if (lim > 0) nt = std::min(nt, lim);
    }
    nt = (int)std::min<int64_t>(nt, n);
    if (nt <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::exception_ptr err;
    std::mutex mu;
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k)
        th.emplace_back([&] {
            try {
                for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                if (!err) err = std::current_exception();
                next.store(n);
            }
        });
    for (auto &t : th) t.join();
    if (err) std::rethrow_exception(err);
}

// C (m x n) = A (m x k) * B (k x n)
inline void gemm_nn(int m, int n, int k, const double *A, const double *B, double *C)
{
    for (int i = 0; i < m; ++i) {
        double *c = C + (size_t)i * n;
        for (int j = 0; j < n; ++j) c[j] = 0.0;
        for (int p = 0; p < k; ++p) {
            const double a = A[(size_t)i * k + p];
            const double *b = B + (size_t)p * n;
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

// C (m x n) = A (m x k) * B^T, B is n x k
inline void gemm_nt(int m, int n, int k, const double *A, const double *B, double *C)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            const double *a = A + (size_t)i * k, *b = B + (size_t)j * k;
            for (int p = 0; p < k; ++p) s += a[p] * b[p];
            C[(size_t)i * n + j] = s;
        }
}

// C (m x n) = A^T * B, A is k x m, B is k x n
inline void gemm_tn(int m, int n, int k, const double *A, const double *B, double *C)
{
    for (int i = 0; i < m * n; ++i) C[i] = 0.0;
    for (int p = 0; p < k; ++p)
        for (int i = 0; i < m; ++i) {
            const double a = A[(size_t)p * m + i];
            const double *b = B + (size_t)p * n;
            double *c = C + (size_t)i * n;
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
}

// Householder QR of A (m x n): Q (m x r) with orthonormal columns and R (r x n),
// r = min(m, n), A = Q R.
void householder_qr(int m, int n, const double *A, std::vector<double> &Q, std::vector<double> &R);

}  // namespace h2b
