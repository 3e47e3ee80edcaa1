// Host FP64 symmetric eigensolver for the PCA basis (Methodology 2.2: PCA
// before the search tree).  Only the d leading eigenpairs are formed:
//   1. Householder reduction to tridiagonal form T = Q^T C Q (Golub & Van
//      Loan, "Matrix Computations", section 8.3.1), with each step's rank-2
//      update fused into the next step's symmetric matrix-vector product so
//      that the trailing matrix is swept once per step; rows are shared out
//      over host threads;
//   2. the d largest eigenvalues of T by Sturm-sequence bisection
//      (section 8.4.1);
//   3. their eigenvectors by inverse iteration on T (section 8.2.2), with
//      Gram-Schmidt inside clusters of close eigenvalues;
//   4. back-transformation by the stored reflectors, then the sign rule
//      (largest-magnitude entry positive, ties to the lowest index).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

#include "eig.hpp"

namespace pts {

namespace {

class Barrier {
 public:
  explicit Barrier(int n) : n_(n) {}
  void wait() {
    std::unique_lock<std::mutex> lk(m_);
    const uint64_t gen = gen_;
    if (++count_ == n_) {
      count_ = 0;
      ++gen_;
      cv_.notify_all();
    } else {
      cv_.wait(lk, [&] { return gen_ != gen; });
    }
  }

 private:
  std::mutex m_;
  std::condition_variable cv_;
  int n_, count_ = 0;
  uint64_t gen_ = 0;
};

// Householder tridiagonalisation, in place on A (n x n, row-major, full
// symmetric storage).  On return diag[n], off[n-1] hold T; row k of A holds
// the reflector v_k in columns k+1..n-1 and beta[k] its scale, so that
// H_k = I - beta_k v_k v_k^T and Q = H_0 H_1 ... H_{n-3}.
void tridiagonalise(std::vector<double>& A, int n, std::vector<double>& diag, std::vector<double>& off,
                    std::vector<double>& beta, int nthreads) {
  diag.assign(n, 0.0);
  off.assign(std::max(n - 1, 0), 0.0);
  beta.assign(n, 0.0);
  if (n == 1) {
    diag[0] = A[0];
    return;
  }
  std::vector<double> v(n, 0.0), w(n, 0.0), p(n, 0.0);    // current step
  std::vector<double> pv(n, 0.0), pw(n, 0.0);             // pending update of previous step
  bool pending = false;
  nthreads = std::max(1, std::min(nthreads, n / 64));
  Barrier bar(nthreads);
  std::atomic<int> stop{0};
  int k_shared = 0;
  double beta_shared = 0.0;

  // worker: applies the pending update to rows [r0, r1) of the trailing block
  // (rows/cols >= k+1) and computes p[i] = beta * row_i . v for those rows.
  auto sweep_rows = [&](int k, int r0, int r1, double bk) {
    const int j0 = k + 1;
    for (int i = r0; i < r1; ++i) {
      double* row = &A[(size_t)i * n];
      double acc = 0.0;
      if (pending) {
        const double pvi = pv[i], pwi = pw[i];
        for (int j = j0; j < n; ++j) {
          const double a = row[j] - pvi * pw[j] - pwi * pv[j];
          row[j] = a;
          acc += a * v[j];
        }
      } else {
        for (int j = j0; j < n; ++j) acc += row[j] * v[j];
      }
      p[i] = bk * acc;
    }
  };

  auto worker = [&](int tid) {
    for (;;) {
      bar.wait();  // step start
      if (stop.load()) return;
      const int k = k_shared;
      const int m = n - (k + 1);
      const int r0 = k + 1 + (int)((int64_t)m * tid / nthreads);
      const int r1 = k + 1 + (int)((int64_t)m * (tid + 1) / nthreads);
      sweep_rows(k, r0, r1, beta_shared);
      bar.wait();  // step end
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker, t);

  for (int k = 0; k <= n - 3; ++k) {
    double* rk = &A[(size_t)k * n];
    // bring row k up to date (columns k..n-1)
    if (pending) {
      const double pvk = pv[k], pwk = pw[k];
      for (int j = k; j < n; ++j) rk[j] -= pvk * pw[j] + pwk * pv[j];
    }
    diag[k] = rk[k];
    // reflector for x = row k, columns k+1..n-1
    double sig = 0.0;
    for (int j = k + 1; j < n; ++j) sig += rk[j] * rk[j];
    const double nx = std::sqrt(sig);
    double bk = 0.0;
    std::fill(v.begin(), v.end(), 0.0);
    if (nx > 0.0) {
      const double x0 = rk[k + 1];
      const double alpha = (x0 >= 0.0) ? -nx : nx;
      for (int j = k + 1; j < n; ++j) v[j] = rk[j];
      v[k + 1] = x0 - alpha;
      double vv = 0.0;
      for (int j = k + 1; j < n; ++j) vv += v[j] * v[j];
      bk = (vv > 0.0) ? 2.0 / vv : 0.0;
      off[k] = alpha;
    } else {
      off[k] = 0.0;
    }
    beta[k] = bk;
    // sweep: pending update of the trailing rows fused with p = beta * S v
    k_shared = k;
    beta_shared = bk;
    if (nthreads > 1) {
      bar.wait();
      const int m = n - (k + 1);
      sweep_rows(k, k + 1, k + 1 + (int)((int64_t)m / nthreads), bk);
      bar.wait();
    } else {
      sweep_rows(k, k + 1, n, bk);
    }
    // w = p - (beta/2)(p.v) v ; store v in row k
    double pv_dot = 0.0;
    for (int j = k + 1; j < n; ++j) pv_dot += p[j] * v[j];
    const double K = 0.5 * bk * pv_dot;
    std::fill(pw.begin(), pw.end(), 0.0);
    std::fill(pv.begin(), pv.end(), 0.0);
    for (int j = k + 1; j < n; ++j) {
      pw[j] = p[j] - K * v[j];
      pv[j] = v[j];
      rk[j] = v[j];
    }
    pending = bk != 0.0;
    if (!pending) {
      // nothing to apply next step
      std::fill(pw.begin(), pw.end(), 0.0);
    }
  }
  if (nthreads > 1) {
    stop.store(1);
    bar.wait();
    for (auto& t : pool) t.join();
  }
  // last 2x2 block: apply the pending update to rows n-2, n-1
  for (int i = std::max(0, n - 2); i < n; ++i) {
    double* row = &A[(size_t)i * n];
    if (pending)
      for (int j = std::max(0, n - 2); j < n; ++j) row[j] -= pv[i] * pw[j] + pw[i] * pv[j];
  }
  if (n >= 2) {
    diag[n - 2] = A[(size_t)(n - 2) * n + (n - 2)];
    diag[n - 1] = A[(size_t)(n - 1) * n + (n - 1)];
    off[n - 2] = A[(size_t)(n - 2) * n + (n - 1)];
    beta[n - 2] = 0.0;
    beta[n - 1] = 0.0;
  }
}

// number of eigenvalues of T strictly below x (Sturm sequence)
int sturm_count(const std::vector<double>& a, const std::vector<double>& e2, double x, double pivmin) {
  const int n = (int)a.size();
  int cnt = 0;
  double q = a[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = a[i] - x - e2[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// solve (T - lambda I) y = b in place (b -> y), Gaussian elimination with
// partial pivoting on the tridiagonal matrix
void tri_solve(const std::vector<double>& a, const std::vector<double>& e, double lambda, std::vector<double>& b,
               double tiny) {
  const int n = (int)a.size();
  if (n == 1) {
    double d = a[0] - lambda;
    if (std::fabs(d) < tiny) d = tiny;
    b[0] /= d;
    return;
  }
  // U has diagonal u0, superdiagonals u1, u2; multipliers l
  std::vector<double> u0(n), u1(n, 0.0), u2(n, 0.0), l(n, 0.0);
  std::vector<char> swp(n, 0);
  double d = a[0] - lambda, s1 = e[0];
  for (int i = 0; i < n - 1; ++i) {
    // current row i: (d, s1, s2=0) ; next row i+1: (e[i], a[i+1]-lambda, e[i+1])
    const double nd = e[i], nd1 = a[i + 1] - lambda, nd2 = (i + 1 < n - 1) ? e[i + 1] : 0.0;
    if (std::fabs(d) >= std::fabs(nd)) {
      if (std::fabs(d) < tiny) d = tiny;
      const double m = nd / d;
      l[i] = m;
      u0[i] = d;
      u1[i] = s1;
      u2[i] = 0.0;
      d = nd1 - m * s1;
      s1 = nd2;
      swp[i] = 0;
    } else {
      const double m = d / nd;
      l[i] = m;
      u0[i] = nd;
      u1[i] = nd1;
      u2[i] = nd2;
      d = s1 - m * nd1;
      s1 = -m * nd2;
      swp[i] = 1;
    }
  }
  if (std::fabs(d) < tiny) d = tiny;
  u0[n - 1] = d;
  // forward elimination on b
  for (int i = 0; i < n - 1; ++i) {
    if (swp[i]) std::swap(b[i], b[i + 1]);
    b[i + 1] -= l[i] * b[i];
  }
  // back substitution
  b[n - 1] /= u0[n - 1];
  if (n >= 2) b[n - 2] = (b[n - 2] - u1[n - 2] * b[n - 1]) / u0[n - 2];
  for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - u1[i] * b[i + 1] - u2[i] * b[i + 2]) / u0[i];
}

}  // namespace

int eig_sym_top(const double* C, int n, int d, double* evals, double* evecs, int nthreads) {
  if (n <= 0 || d <= 0 || d > n) return -1;
  std::vector<double> A(C, C + (size_t)n * n);
  std::vector<double> a, e, beta;
  if (nthreads <= 0) nthreads = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  tridiagonalise(A, n, a, e, beta, nthreads);

  // scale and Gershgorin interval
  double tnorm = 0.0, lo = 0.0, hi = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(e[i]) : 0.0);
    tnorm = std::max(tnorm, std::fabs(a[i]) + r);
    lo = (i == 0) ? a[i] - r : std::min(lo, a[i] - r);
    hi = (i == 0) ? a[i] + r : std::max(hi, a[i] + r);
  }
  if (tnorm == 0.0) tnorm = 1.0;
  std::vector<double> e2(std::max(n - 1, 0));
  for (int i = 0; i < n - 1; ++i) e2[i] = e[i] * e[i];
  const double eps = 2.220446049250313e-16;
  const double pivmin = std::max(1e-300, eps * eps * tnorm * tnorm * 1e-10);
  lo -= 2 * eps * tnorm + pivmin;
  hi += 2 * eps * tnorm + pivmin;

  // bisection: k-th smallest for k = n-1 .. n-d (descending output)
  std::vector<double> lam(d);
  for (int j = 0; j < d; ++j) {
    const int k = n - 1 - j;
    double l = lo, h = hi;
    for (int it = 0; it < 200 && h - l > 2 * eps * std::max(std::fabs(l), std::fabs(h)) + pivmin; ++it) {
      const double mid = 0.5 * (l + h);
      if (sturm_count(a, e2, mid, pivmin) <= k)
        l = mid;
      else
        h = mid;
    }
    lam[j] = 0.5 * (l + h);
  }

  // inverse iteration
  std::vector<std::vector<double>> Y(d, std::vector<double>(n));
  const double sep = 1e-3 * tnorm;
  int cluster_start = 0;
  uint64_t rs = 0x9E3779B97F4A7C15ull;
  for (int j = 0; j < d; ++j) {
    if (j > 0 && std::fabs(lam[j - 1] - lam[j]) > sep) cluster_start = j;
    double shift = lam[j];
    // separate shifts of (numerically) equal eigenvalues inside a cluster
    for (int t = cluster_start; t < j; ++t)
      if (std::fabs(lam[t] - shift) < 10 * eps * tnorm) shift -= 10 * eps * tnorm;
    std::vector<double>& y = Y[j];
    for (int i = 0; i < n; ++i) {
      rs ^= rs << 13;
      rs ^= rs >> 7;
      rs ^= rs << 17;
      y[i] = ((double)(rs >> 11) / 9007199254740992.0) - 0.5;
    }
    for (int it = 0; it < 4; ++it) {
      tri_solve(a, e, shift, y, pivmin + eps * tnorm);
      for (int t = cluster_start; t < j; ++t) {  // orthogonalise within the cluster
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += y[i] * Y[t][i];
        for (int i = 0; i < n; ++i) y[i] -= dot * Y[t][i];
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += y[i] * y[i];
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) {
        y.assign(n, 0.0);
        y[j % n] = 1.0;
        nrm = 1.0;
      }
      for (int i = 0; i < n; ++i) y[i] /= nrm;
    }
  }

  // back-transform: x = H_0 H_1 ... H_{n-3} y
  for (int j = 0; j < d; ++j) {
    std::vector<double>& y = Y[j];
    for (int k = n - 3; k >= 0; --k) {
      const double bk = beta[k];
      if (bk == 0.0) continue;
      const double* vk = &A[(size_t)k * n];
      double dot = 0.0;
      for (int i = k + 1; i < n; ++i) dot += vk[i] * y[i];
      dot *= bk;
      for (int i = k + 1; i < n; ++i) y[i] -= dot * vk[i];
    }
    // sign rule
    int im = 0;
    double am = -1.0;
    for (int i = 0; i < n; ++i)
      if (std::fabs(y[i]) > am) {
        am = std::fabs(y[i]);
        im = i;
      }
    if (y[im] < 0)
      for (int i = 0; i < n; ++i) y[i] = -y[i];
    for (int i = 0; i < n; ++i) evecs[(size_t)i * d + j] = y[i];
    evals[j] = lam[j];
  }
  return 0;
}

}  // namespace pts
