// Setup of the Hessenberg form of the velocity-space systems (FP64, host).
//
// In the spherical-harmonic basis (eq. f_expansion, unknowns ordered l-major)
// the V system of eq. (vspace_batched_system) at a point with field E is
//     (B - s A_h) u = b,   B = I - dt n0 C_h,  s = dt E,
// where C_h is block diagonal in l (the collision operator does not couple
// harmonics), so B is cheap to invert block by block.  With K = B^-1 A_h reduced
// once by orthogonal similarity to upper Hessenberg form, K = Q H Q^T,
//     u = Q (I - s H)^-1 W b,   W = Q^T B^-1,
// and each point's solve costs O(n^2) instead of the O(n^3) of a factorization
// (the frequency-response form of Laub, IEEE TAC 1981, for a pencil whose first
// matrix is well conditioned).  The reduction is the Householder one
// (Golub and Van Loan, Matrix Computations, the Hessenberg reduction algorithm),
// backward stable like the transforms that follow.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <thread>
#include <vector>

#include "assemble.h"
#include "hessenberg.h"

namespace bte {
namespace {

// A fixed team of threads running one function per phase, with a barrier
// between phases (the reduction has two dependent updates per column).
class Team {
 public:
  explicit Team(int n) : n_(std::max(1, n)) {
    for (int t = 1; t < n_; ++t) pool_.emplace_back([this, t] { loop(t); });
  }
  ~Team() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& th : pool_) th.join();
  }
  int size() const { return n_; }
  // runs f(t) on every thread t = 0..size()-1 and returns when all are done
  void run(const std::function<void(int)>& f) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &f;
      left_ = n_ - 1;
      ++gen_;
    }
    cv_.notify_all();
    f(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [this] { return left_ == 0; });
    fn_ = nullptr;
  }

 private:
  void loop(int t) {
    unsigned long seen = 0;
    for (;;) {
      const std::function<void(int)>* f = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        if (stop_) return;
        f = fn_;
      }
      (*f)(t);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (--left_ == 0) done_.notify_one();
      }
    }
  }
  int n_;
  std::vector<std::thread> pool_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* fn_ = nullptr;
  unsigned long gen_ = 0;
  int left_ = 0;
  bool stop_ = false;
};

inline void split(int lo, int hi, int t, int nt, int* a, int* b) {
  const int len = hi - lo;
  *a = lo + static_cast<int>(static_cast<long long>(len) * t / nt);
  *b = lo + static_cast<int>(static_cast<long long>(len) * (t + 1) / nt);
}

// LU with partial pivoting of a small dense block (row-major m x m), in place;
// then X <- A^-1 X for X row-major m x ncol.
void lu_solve_block(std::vector<double> A, int m, double* X, int ncol, int ldx) {
  std::vector<int> piv(m);
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (std::fabs(A[i * m + k]) > std::fabs(A[p * m + k])) p = i;
    if (A[p * m + k] == 0.0) throw std::runtime_error("singular collision block");
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < m; ++j) std::swap(A[k * m + j], A[p * m + j]);
    for (int i = k + 1; i < m; ++i) {
      const double l = A[i * m + k] / A[k * m + k];
      A[i * m + k] = l;
      for (int j = k + 1; j < m; ++j) A[i * m + j] -= l * A[k * m + j];
    }
  }
  for (int k = 0; k < m; ++k)
    if (piv[k] != k)
      for (int j = 0; j < ncol; ++j) std::swap(X[(size_t)k * ldx + j], X[(size_t)piv[k] * ldx + j]);
  for (int i = 1; i < m; ++i)
    for (int k = 0; k < i; ++k) {
      const double l = A[i * m + k];
      if (l != 0.0)
        for (int j = 0; j < ncol; ++j) X[(size_t)i * ldx + j] -= l * X[(size_t)k * ldx + j];
    }
  for (int i = m - 1; i >= 0; --i) {
    for (int k = i + 1; k < m; ++k) {
      const double u = A[i * m + k];
      if (u != 0.0)
        for (int j = 0; j < ncol; ++j) X[(size_t)i * ldx + j] -= u * X[(size_t)k * ldx + j];
    }
    const double d = A[i * m + i];
    for (int j = 0; j < ncol; ++j) X[(size_t)i * ldx + j] /= d;
  }
}

}  // namespace

void hessenberg_reduce(std::vector<double>& K, int n, std::vector<double>* Qout, int nthreads) {
  Team team(nthreads);
  const int nt = team.size();
  std::vector<double> V((size_t)n * n, 0.0), beta(n, 0.0);   // reflector k in V[k][k+1..n)
  for (int k = 0; k + 2 < n; ++k) {
    // Householder vector v (v[0] = 1) with (I - beta v v^T) x = alpha e_1, x = K[k+1.., k]
    double* v = V.data() + (size_t)k * n;
    double sig = 0.0;
    for (int i = k + 2; i < n; ++i) sig += K[(size_t)i * n + k] * K[(size_t)i * n + k];
    const double x0 = K[(size_t)(k + 1) * n + k];
    if (sig == 0.0) {
      beta[k] = 0.0;
      continue;
    }
    const double mu = std::sqrt(x0 * x0 + sig);
    const double v0 = (x0 <= 0.0) ? x0 - mu : -sig / (x0 + mu);
    beta[k] = 2.0 * v0 * v0 / (sig + v0 * v0);
    v[k + 1] = 1.0;
    for (int i = k + 2; i < n; ++i) v[i] = K[(size_t)i * n + k] / v0;
    const double b = beta[k];
    // left: K[k+1.., k..] -= b v (v^T K[k+1.., k..]), by column ranges
    team.run([&](int t) {
      int j0, j1;
      split(k, n, t, nt, &j0, &j1);
      if (j0 >= j1) return;
      std::vector<double> acc(j1 - j0, 0.0);
      for (int i = k + 1; i < n; ++i) {
        const double vi = v[i];
        const double* row = K.data() + (size_t)i * n;
        for (int j = j0; j < j1; ++j) acc[j - j0] += vi * row[j];
      }
      for (int i = k + 1; i < n; ++i) {
        const double s = b * v[i];
        double* row = K.data() + (size_t)i * n;
        for (int j = j0; j < j1; ++j) row[j] -= s * acc[j - j0];
      }
    });
    // right: K[.., k+1..] -= b (K[.., k+1..] v) v^T, by row ranges
    team.run([&](int t) {
      int i0, i1;
      split(0, n, t, nt, &i0, &i1);
      for (int i = i0; i < i1; ++i) {
        double* row = K.data() + (size_t)i * n;
        double s = 0.0;
        for (int j = k + 1; j < n; ++j) s += row[j] * v[j];
        s *= b;
        for (int j = k + 1; j < n; ++j) row[j] -= s * v[j];
      }
    });
    // the reflector maps x to mu e_1 (either sign of x0, by the choice of v0)
    K[(size_t)(k + 1) * n + k] = mu;
    for (int i = k + 2; i < n; ++i) K[(size_t)i * n + k] = 0.0;
  }
  // Q = P_0 P_1 ... P_{n-3}, accumulated backwards: Q <- P_k Q on rows/cols k+1..
  std::vector<double>& Q = *Qout;
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    if (beta[k] == 0.0) continue;
    const double* v = V.data() + (size_t)k * n;
    const double b = beta[k];
    team.run([&](int t) {
      int j0, j1;
      split(k + 1, n, t, nt, &j0, &j1);
      if (j0 >= j1) return;
      std::vector<double> acc(j1 - j0, 0.0);
      for (int i = k + 1; i < n; ++i) {
        const double vi = v[i];
        const double* row = Q.data() + (size_t)i * n;
        for (int j = j0; j < j1; ++j) acc[j - j0] += vi * row[j];
      }
      for (int i = k + 1; i < n; ++i) {
        const double s = b * v[i];
        double* row = Q.data() + (size_t)i * n;
        for (int j = j0; j < j1; ++j) row[j] -= s * acc[j - j0];
      }
    });
  }
}

void hessenberg_setup(const HostOps& H, double n0, double dt, int nthreads, HessForm* out) {
  const int nr = H.nr, nl = H.nl, n = H.nh;
  // K = B^-1 A_h with B = I - dt n0 C_h block diagonal in l (nr x nr blocks)
  std::vector<double> K((size_t)n * n), Binv((size_t)n * n, 0.0);
  for (size_t i = 0; i < K.size(); ++i) K[i] = H.Ah[i];
  for (int l = 0; l < nl; ++l) {
    std::vector<double> blk((size_t)nr * nr);
    for (int r = 0; r < nr; ++r)
      for (int c = 0; c < nr; ++c)
        blk[r * nr + c] = (r == c ? 1.0 : 0.0) - dt * n0 * H.Ch[(size_t)(l * nr + r) * n + l * nr + c];
    for (int r = 0; r < nr; ++r) Binv[(size_t)(l * nr + r) * n + l * nr + r] = 1.0;
    lu_solve_block(blk, nr, K.data() + (size_t)l * nr * n, n, n);              // rows of block l of K
    lu_solve_block(blk, nr, Binv.data() + (size_t)l * nr * n + l * nr, nr, n);  // its block of B^-1
  }
  hessenberg_reduce(K, n, &out->Q, nthreads);
  out->n = n;
  // H column-major (each column read contiguously by the solve); entries below
  // the subdiagonal are exactly zero
  out->Hc.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c)
    for (int r = 0; r <= std::min(c + 1, n - 1); ++r) out->Hc[(size_t)c * n + r] = K[(size_t)r * n + c];
  // W = Q^T B^-1: column block l of W is Q^T's column block l times the nr x nr block of B^-1
  out->W.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < nl; ++l)
      for (int c = 0; c < nr; ++c) {
        double s = 0.0;
        for (int r = 0; r < nr; ++r) s += out->Q[(size_t)(l * nr + r) * n + i] * Binv[(size_t)(l * nr + r) * n + l * nr + c];
        out->W[(size_t)i * n + l * nr + c] = s;
      }
}

}  // namespace bte
