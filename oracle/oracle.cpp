// oracle.cpp -- plain FP64 CPU reference for recursive spectral bisection.
//
// TEST INFRASTRUCTURE ONLY: the GPU library never includes, links or calls
// this file.  It is deliberately simple (maps, explicit loops) so that each
// function can be checked against the paper by eye.  Element loops may run
// on several OpenMP threads; sums keep one fixed order (fixed_sum), so the
// thread count never changes a result.
//
// Readings where the paper is silent (each is also stated where it is used):
//  * a vertex id repeated inside one element counts once (set semantics);
//  * "face connected" means sharing at least nv/2 vertex ids;
//  * the start vector is r_i = U[-1, 1) from splitmix64(seed, gid_i);
//  * the ones vector u0 = 1/sqrt(n) is kept in the reorthogonalisation basis;
//  * two classical Gram-Schmidt passes per Lanczos step;
//  * convergence when ||L y - rho y||_2 <= tol * rho (rho the Rayleigh quotient
//    of the Ritz vector); explicit restart from the Ritz vector, or thick
//    restart keeping the smallest Ritz pairs; at most max_restarts restarts;
//  * canonical sign: the first element (in global-id order) whose |y| is at
//    least 1e-3 max|y| gets y <= 0;
//  * ties in the sort broken by global id, -0.0 before +0.0;
//  * low side gets P_L = floor(P/2) parts and floor(n P_L / P) elements;
//  * disconnected subgraphs: components ordered by smallest global id go
//    whole to one side; only the component that straddles the target count
//    is cut, by its own Fiedler vector.
#include "oracle.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <unordered_map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef std::vector<double> Vec;

// ---------------------------------------------------------------------------
// Threads (optional).  Loops over vector elements may run on several threads;
// every sum over elements is taken in one fixed order: consecutive chunks of
// kSumChunk terms are summed one by one, then the chunk sums in chunk order.
// Chunk boundaries do not depend on the thread count, so one thread and many
// threads give the same bits.  Element-wise loops have no order to keep.
// ---------------------------------------------------------------------------
constexpr int64_t kSumChunk = 4096;
// element loops run threaded only above this length (thread start-up costs
// more than it saves on short vectors)
constexpr int64_t kThreadMin = 16384;

template <class F>
double fixed_sum(int64_t n, F term) {
  const int64_t nc = (n + kSumChunk - 1) / kSumChunk;
  std::vector<double> part((size_t)std::max<int64_t>(nc, 1), 0.0);
#pragma omp parallel for schedule(static) if (nc >= 4)
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t lo = c * kSumChunk, hi = std::min(n, lo + kSumChunk);
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += term(i);
    part[(size_t)c] = s;
  }
  double s = 0.0;
  for (int64_t c = 0; c < nc; ++c) s += part[(size_t)c];
  return s;
}

// ---------------------------------------------------------------------------
// Graph held as adjacency lists (sorted by neighbour index).
// ---------------------------------------------------------------------------
struct Graph {
  int64_t n = 0;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> adj;  // (neighbour, weight)
};

// Edge weight from the number s of vertex ids two elements share
// (Sec. 2: weight = shared vertices, 1/2/4 for hexes; Sec. 4 unweighted
// Laplacian: unit weight; face graph: sharing at least half of the vertices).
int weight_of(int32_t graph, int s, int nv) {
  if (graph == ORC_GRAPH_WEIGHTED) return s;
  if (graph == ORC_GRAPH_UNIT) return 1;
  return (s >= nv / 2) ? 1 : 0;
}

// Dual graph (Sec. 2): vertex = element, edge = elements sharing a mesh vertex.
// Built by a vertex -> elements map and per-element neighbour counting.
Graph build_dual_graph(int64_t nelem, int nv, const int64_t *ids, int32_t graph) {
  std::unordered_map<int64_t, std::vector<int32_t>> elems_of_vertex;
  std::vector<std::vector<int64_t>> distinct(nelem);
  for (int64_t e = 0; e < nelem; ++e) {
    std::set<int64_t> s(ids + e * nv, ids + (e + 1) * nv);
    distinct[e].assign(s.begin(), s.end());
    for (int64_t v : distinct[e]) elems_of_vertex[v].push_back((int32_t)e);
  }
  Graph g;
  g.n = nelem;
  g.adj.resize(nelem);
  for (int64_t e = 0; e < nelem; ++e) {
    std::map<int32_t, int> shared;  // neighbour -> number of shared vertex ids
    for (int64_t v : distinct[e])
      for (int32_t j : elems_of_vertex[v])
        if (j != e) shared[j] += 1;
    for (auto &kv : shared) {
      int w = weight_of(graph, kv.second, nv);
      if (w > 0) g.adj[e].push_back({kv.first, w});
    }
  }
  return g;
}

// y = L x with L = D - A (Sec. 4): l_ii = sum_j w_ij, l_ij = -w_ij.
void apply_laplacian(const Graph &g, const Vec &x, Vec &y) {
#pragma omp parallel for schedule(static) if (g.n >= kThreadMin)
  for (int64_t i = 0; i < g.n; ++i) {
    double d = 0.0, ax = 0.0;
    for (auto &nw : g.adj[i]) {
      d += nw.second;
      ax += nw.second * x[nw.first];
    }
    y[i] = d * x[i] - ax;
  }
}

double dot(const Vec &a, const Vec &b) {
  const double *pa = a.data(), *pb = b.data();
  return fixed_sum((int64_t)a.size(), [=](int64_t i) { return pa[i] * pb[i]; });
}

double norm2(const Vec &a) { return std::sqrt(dot(a, a)); }

// splitmix64 (Steele, Lea, Flood 2014): output for counter c of the stream
// started at seed is mix(seed + c * golden_gamma).
uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + counter * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double start_value(uint64_t seed, int64_t gid) {
  uint64_t z = splitmix64_at(seed, (uint64_t)gid + 1);
  return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// ---------------------------------------------------------------------------
// Smallest eigenpair of a symmetric tridiagonal matrix: Sturm-sequence
// bisection for the eigenvalue, inverse iteration for the eigenvector.
// ---------------------------------------------------------------------------

// Number of eigenvalues of T strictly below x (signs of the pivots of the
// LDL^T factorisation of T - x I).
int sturm_count(int k, const double *a, const double *b, double x) {
  int count = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    double off = (i == 0) ? 0.0 : b[i] * b[i] / q;
    q = (a[i] - x) - off;
    if (q == 0.0) q = -1e-300;  // a zero pivot is taken as a tiny negative
    if (q < 0.0) ++count;
  }
  return count;
}

// Solve (T - s I) z = r for tridiagonal T by Gaussian elimination with
// partial pivoting (the system is nearly singular in inverse iteration).
void tridiag_shifted_solve(int k, const double *a, const double *b, double s, Vec &z) {
  // Row i of the band: [l_i, d_i, u_i, u2_i] after pivoting.
  Vec d(k), u(k, 0.0), u2(k, 0.0), l(k, 0.0), rhs = z;
  for (int i = 0; i < k; ++i) {
    d[i] = a[i] - s;
    if (i + 1 < k) u[i] = b[i + 1];
    if (i > 0) l[i] = b[i];
  }
  // a zero pivot is replaced by a perturbation of the size of rounding
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(a[i]) + (i ? std::fabs(b[i]) : 0.0));
  double tiny = std::max(scale, 1e-300) * 2.220446049250313e-16;
  for (int i = 0; i + 1 < k; ++i) {
    // candidate pivot rows i (d[i], u[i], u2[i]) and i+1 (l[i+1], d[i+1], u[i+1])
    if (std::fabs(l[i + 1]) > std::fabs(d[i])) {
      std::swap(d[i], l[i + 1]);
      std::swap(u[i], d[i + 1]);
      std::swap(u2[i], u[i + 1]);
      std::swap(rhs[i], rhs[i + 1]);
    }
    if (d[i] == 0.0) d[i] = tiny;
    double f = l[i + 1] / d[i];
    d[i + 1] -= f * u[i];
    u[i + 1] -= f * u2[i];
    rhs[i + 1] -= f * rhs[i];
    l[i + 1] = 0.0;
  }
  if (d[k - 1] == 0.0) d[k - 1] = tiny;
  for (int i = k - 1; i >= 0; --i) {
    double v = rhs[i];
    if (i + 1 < k) v -= u[i] * rhs[i + 1];
    if (i + 2 < k) v -= u2[i] * rhs[i + 2];
    rhs[i] = v / d[i];
  }
  z = rhs;
}

int tridiag_smallest(int k, const double *a, const double *b, double thr, double *theta, Vec &t) {
  if (k <= 0) return -1;
  // Gershgorin interval
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    double r = 0.0;
    if (i > 0) r += std::fabs(b[i]);
    if (i + 1 < k) r += std::fabs(b[i + 1]);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  // Eigenvalues below thr are spurious null modes and skipped: target the
  // (c0+1)-th smallest eigenvalue, c0 = count below thr.
  int c0 = sturm_count(k, a, b, thr);
  if (c0 >= k) return -1;
  int target = c0 + 1;
  lo = std::max(lo, thr);
  hi = hi + 1e-12 * std::fabs(hi) + 1e-300;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(k, a, b, mid) >= target) hi = mid; else lo = mid;
  }
  double th = 0.5 * (lo + hi);
  *theta = th;
  // inverse iteration from a fixed vector
  t.assign(k, 1.0);
  for (int it = 0; it < 4; ++it) {
    tridiag_shifted_solve(k, a, b, th, t);
    double big = 0.0;
    for (double v : t) big = std::max(big, std::fabs(v));
    for (double &v : t) v /= big;
    double nrm = 0.0;
    for (double v : t) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double &v : t) v /= nrm;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Fiedler pair on a connected graph (one component), Sec. 6 and Sec. 7.
// gid[i]: global id of local vertex i (start vector, sign rule).
// ---------------------------------------------------------------------------

// Remove the ones-vector component: x <- x - (u0^T x) u0 with u0 = 1/sqrt(n).
void deflate_ones(Vec &x) {
  const int64_t n = (int64_t)x.size();
  double *px = x.data();
  double mean = fixed_sum(n, [=](int64_t i) { return px[i]; });
  mean /= (double)n;
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
  for (int64_t i = 0; i < n; ++i) px[i] -= mean;
}

void normalize(Vec &x) {
  const int64_t n = (int64_t)x.size();
  double *px = x.data();
  const double nr = norm2(x);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
  for (int64_t i = 0; i < n; ++i) px[i] /= nr;
}

// Canonical sign: the first element in global-id order whose magnitude is at
// least 1e-3 of the largest gets a non-positive value.
void canonical_sign(Vec &y, const std::vector<int64_t> &gid) {
  double ymax = 0.0;
  for (double v : y) ymax = std::max(ymax, std::fabs(v));
  int64_t best = -1;
  for (size_t i = 0; i < y.size(); ++i)
    if (std::fabs(y[i]) >= 1e-3 * ymax && (best < 0 || gid[i] < gid[best])) best = (int64_t)i;
  if (best >= 0 && y[best] > 0.0)
    for (double &v : y) v = -v;
}

double residual_norm(const Graph &g, const Vec &y, double theta, int64_t &matvecs) {
  Vec ly(g.n);
  apply_laplacian(g, y, ly);
  ++matvecs;
  const double *pl = ly.data(), *py = y.data();
  const double s = fixed_sum(g.n, [=](int64_t i) {
    const double r = pl[i] - theta * py[i];
    return r * r;
  });
  return std::sqrt(s);
}

double rayleigh(const Graph &g, const Vec &y, int64_t &matvecs) {
  Vec ly(g.n);
  apply_laplacian(g, y, ly);
  ++matvecs;
  return dot(y, ly) / dot(y, y);
}

// Eigen-decomposition of a symmetric k x k matrix (row-major) by the cyclic
// Jacobi method (Golub & Van Loan, Sec. 8.5): rotations in every (p, q)
// plane until the off-diagonal part is at rounding level.  Output: the
// eigenvalues in ascending order and the eigenvectors as columns of V.
void jacobi_eigen(int k, Vec A, Vec &ev, Vec &V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  double fro = 0.0;
  for (double v : A) fro += v * v;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += 2.0 * A[(size_t)p * k + q] * A[(size_t)p * k + q];
    if (std::sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
    for (int p = 0; p < k; ++p) {
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        // 2x2 symmetric Schur decomposition: c, s with tan = t
        const double tau = (A[(size_t)q * k + q] - A[(size_t)p * k + p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        // A <- J^T A J with J the rotation in the (p, q) plane
        for (int r = 0; r < k; ++r) {
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = c * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = c * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = c * vrp - sn * vrq;
          V[(size_t)r * k + q] = sn * vrp + c * vrq;
        }
      }
    }
  }
  // sort ascending (stable selection on the diagonal)
  std::vector<int> order(k);
  for (int i = 0; i < k; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return A[(size_t)a * k + a] < A[(size_t)b * k + b];
  });
  Vec V2((size_t)k * k);
  ev.assign(k, 0.0);
  for (int c = 0; c < k; ++c) {
    ev[c] = A[(size_t)order[c] * k + order[c]];
    for (int r = 0; r < k; ++r) V2[(size_t)r * k + c] = V[(size_t)r * k + order[c]];
  }
  V.swap(V2);
}

// Restarted Lanczos with full reorthogonalisation (Sec. 6).
//
// keep = 0: explicit restart -- every cycle starts a new Krylov space from
// the current Ritz vector (the scheme the paper describes).
// keep > 0: thick restart (Wu and Simon, the Lanczos variant the paper
// cites in Sec. 6): the cycle keeps the `keep` smallest Ritz pairs
// (theta_i, y_i) and continues from the last Lanczos residual direction
// q = w / beta.  The projected matrix of the next cycle is then
//   [ diag(theta)  s        ]
//   [ s^T          alpha ... ]  (tridiagonal from there on),
// with s_i = beta * (last component of the i-th Ritz vector of the small
// problem).  The first kept vector is the Ritz vector used for the
// convergence test, re-projected against the ones vector and normalised.
// A cycle that ends by breakdown restarts explicitly.
// Warm start (an addition; the paper leaves the start vector open): a child
// subgraph's solve starts from its parent's second Ritz vector, scaled to
// unit root-mean-square on the parent's component, plus kWarmNoise times the
// usual random start; elements without such a value take the random start.
constexpr double kWarmNoise = 0.1;

// Second Ritz pair of the last cycle (thick restart only): the Ritz vector
// next to the Fiedler one and both Ritz values, for the sweep over the pair.
struct SecondPair {
  bool ok = false;
  Vec y2;
  double theta1 = 0.0, theta2 = 0.0;
};

// Warm start values by global id (carried from a parent bisection).
typedef std::unordered_map<int64_t, double> WarmMap;

int lanczos_fiedler(const Graph &g, const std::vector<int64_t> &gid, const orc_opts &o, Vec &y,
                    double &lambda, orc_info &info, SecondPair *second = nullptr,
                    const WarmMap *warm = nullptr) {
  const int64_t n = g.n;
  const double u0 = 1.0 / std::sqrt((double)n);
  Vec q(n);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
  for (int64_t i = 0; i < n; ++i) {
    q[i] = start_value(o.seed, gid[i]);
    if (warm) {
      auto it = warm->find(gid[i]);
      if (it != warm->end()) q[i] = it->second + kWarmNoise * q[i];
    }
  }
  deflate_ones(q);
  normalize(q);
  const int m = std::max(1, o.lanczos_m);
  const int keep = std::max(0, o.lanczos_keep);
  // two steps at a time only on graphs of more than 4 m elements: a cycle
  // can exhaust the Krylov space of a smaller one (at most m + 1 elements,
  // or fewer distinct eigenvalues than m), and one step at a time meets the
  // breakdown there with both Gram-Schmidt passes behind it
  const bool pairs = o.lanczos_s == 2 && n > 4 * (int64_t)m;
  int converged = 0;
  double theta = 0.0, res = 0.0;
  y = q;
  std::vector<Vec> Y;         // kept Ritz vectors (thick restart)
  Vec th_keep, s_keep;        // their Ritz values and couplings to q
  for (int cycle = 0; cycle <= o.max_restarts; ++cycle) {
    const int nk = (int)Y.size();
    std::vector<Vec> Q(Y);
    Q.push_back(q);
    Vec H((size_t)m * m, 0.0);  // projected matrix (thick restart)
    std::vector<double> alpha(nk, 0.0), beta(nk + 1, 0.0);  // beta[j] couples Q[j-1], Q[j]
    double tnorm = 0.0;
    for (int i = 0; i < nk; ++i) {
      H[(size_t)i * m + i] = th_keep[i];
      H[(size_t)i * m + nk] = H[(size_t)nk * m + i] = s_keep[i];
      tnorm = std::max(tnorm, std::fabs(th_keep[i]) + std::fabs(s_keep[i]));
    }
    Vec w(n);
    double last_b = 0.0;
    bool breakdown = false;
    for (int j = nk; j < m; ++j) {
      if (pairs && j >= 2 && j + 1 < m) {
        // Two steps from one block (step j+1 and j+2 in the paper's
        // numbering): K = [L q_j, L^2 q_j], two classical Gram-Schmidt
        // passes of both columns against [u0, Q[0..j]], then Cholesky QR of
        // the remainder W = [w1, w2] = [q_{j+1}, q_{j+2}] [[R00, R01], [0, R11]].
        // Projected matrix: alpha_j = q_j^T L q_j (coefficient of L q_j on
        // q_j), beta_{j+1} = R00, and, since L q_{j+1} = (L^2 q_j - L V h1) / R00
        // and only q_j of the old basis couples to q_{j+1},
        // alpha_{j+1} = q_{j+1}^T L q_{j+1} = R01 / R00 - alpha_j,
        // beta_{j+2} = q_{j+2}^T L q_{j+1} = R11 / R00.
        Vec w2(n);
        apply_laplacian(g, Q[j], w);
        apply_laplacian(g, w, w2);
        info.matvecs += 2;
        double a = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
          for (Vec *col : {&w, &w2}) {
            const double *pw = col->data();
            const double h0 = fixed_sum(n, [=](int64_t i) { return u0 * pw[i]; });
            std::vector<double> h(j + 1);
            for (int k2 = 0; k2 <= j; ++k2) h[k2] = dot(Q[k2], *col);
            Vec &c = *col;
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
            for (int64_t i = 0; i < n; ++i) {
              double s = h0 * u0;
              for (int k2 = 0; k2 <= j; ++k2) s += h[k2] * Q[k2][i];
              c[i] -= s;
            }
            if (col == &w) a += h[j];
          }
        }
        const double g00 = dot(w, w), g01 = dot(w, w2), g11 = dot(w2, w2);
        const double r00 = std::sqrt(g00);
        alpha.push_back(a);
        H[(size_t)j * m + j] = a;
        tnorm = std::max(tnorm, std::fabs(a) + r00 + (j == nk ? 0.0 : beta[j]));
        if (r00 <= 1e-12 * tnorm) {  // breakdown after step j+1
          last_b = r00;
          breakdown = true;
          break;
        }
        const double r01 = g01 / r00;
        const double r11 = std::sqrt(std::max(g11 - r01 * r01, 0.0));
        const double a1 = r01 / r00 - a, b1 = r00, b2 = r11 / r00;
        beta.push_back(b1);
        H[(size_t)j * m + j + 1] = H[(size_t)(j + 1) * m + j] = b1;
        Vec qa(n);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
        for (int64_t i = 0; i < n; ++i) qa[i] = w[i] / r00;
        Q.push_back(qa);
        alpha.push_back(a1);
        H[(size_t)(j + 1) * m + j + 1] = a1;
        tnorm = std::max(tnorm, std::fabs(a1) + b2 + b1);
        // the next direction, unnormalised with norm beta_{j+2}:
        // (w2 - R01 q_{j+1}) / R00
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
        for (int64_t i = 0; i < n; ++i) w[i] = (w2[i] - r01 * qa[i]) / r00;
        last_b = b2;
        ++j;
        if (j == m - 1) break;
        // R11^2 = g11 - R01^2 is the difference of two numbers of size
        // ||w2||^2, so R11 carries a relative error of about u ||w2||^2 /
        // R11^2.  Below 1e-8 ||w2||^2 (the second column nearly in the span
        // of the first and the basis: the Krylov space is exhausted or
        // nearly so) q_{j+2} = w / beta_{j+2} would no longer be of unit
        // norm to working accuracy, and the cycle ends after step j+1 as at
        // a breakdown.
        if (b2 <= 1e-12 * tnorm || g11 - r01 * r01 <= 1e-8 * g11) {
          breakdown = true;
          break;
        }
        beta.push_back(b2);
        H[(size_t)j * m + j + 1] = H[(size_t)(j + 1) * m + j] = b2;
        Vec qb(n);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
        for (int64_t i = 0; i < n; ++i) qb[i] = w[i] / b2;
        Q.push_back(qb);
        continue;
      }
      apply_laplacian(g, Q[j], w);
      ++info.matvecs;
      double a = dot(Q[j], w);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
      for (int64_t i = 0; i < n; ++i) {
        w[i] -= a * Q[j][i];
        if (j == nk)
          for (int c = 0; c < nk; ++c) w[i] -= s_keep[c] * Y[c][i];
        else
          w[i] -= beta[j] * Q[j - 1][i];
      }
      // two classical Gram-Schmidt passes against [u0, Q[0..j]]
      for (int pass = 0; pass < 2; ++pass) {
        const double *pw = w.data();
        const double h0 = fixed_sum(n, [=](int64_t i) { return u0 * pw[i]; });
        std::vector<double> h(j + 1);
        for (int k = 0; k <= j; ++k) h[k] = dot(Q[k], w);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
        for (int64_t i = 0; i < n; ++i) {
          double s = h0 * u0;
          for (int k = 0; k <= j; ++k) s += h[k] * Q[k][i];
          w[i] -= s;
        }
        a += h[j];
      }
      alpha.push_back(a);
      H[(size_t)j * m + j] = a;
      double b = norm2(w);
      tnorm = std::max(tnorm, std::fabs(a) + b + (j == nk ? 0.0 : beta[j]));
      last_b = b;
      if (j == m - 1) break;
      if (b <= 1e-12 * tnorm) {
        breakdown = true;
        break;
      }
      beta.push_back(b);
      H[(size_t)j * m + j + 1] = H[(size_t)(j + 1) * m + j] = b;
      Vec qn(n);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
      for (int64_t i = 0; i < n; ++i) qn[i] = w[i] / b;
      Q.push_back(qn);
    }
    const int k = (int)Q.size();
    const double thr = 1e-10 * tnorm;
    Vec t;                    // Ritz coefficients of the vector tested for convergence
    Vec ev, EV;               // all eigenpairs of H (thick restart)
    int first = 0;
    if (keep == 0) {
      if (tridiag_smallest(k, alpha.data(), beta.data(), thr, &theta, t) != 0) return -5;
    } else {
      Vec Hk((size_t)k * k);
      for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) Hk[(size_t)r * k + c] = H[(size_t)r * m + c];
      jacobi_eigen(k, Hk, ev, EV);
      while (first < k && ev[first] < thr) ++first;
      if (first >= k) return -5;
      theta = ev[first];
      t.assign(k, 0.0);
      for (int r = 0; r < k; ++r) t[r] = EV[(size_t)r * k + first];
    }
    // Ritz vector y = Q t, re-projected against the ones vector and normalised
    y.assign(n, 0.0);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < k; ++c) y[i] += t[c] * Q[c][i];
    deflate_ones(y);
    normalize(y);
    // residual against the Rayleigh quotient rho of the Ritz vector
    double rho = rayleigh(g, y, info.matvecs);
    res = residual_norm(g, y, rho, info.matvecs);
    info.cycles = cycle + 1;
    if (second) {
      second->ok = (keep >= 2 && first + 1 < k && std::min(keep, k - 1) >= 2);
      if (second->ok) {
        second->theta1 = ev[first];
        second->theta2 = ev[first + 1];
        second->y2.assign(n, 0.0);
        Vec &y2 = second->y2;
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
        for (int64_t i = 0; i < n; ++i)
          for (int c = 0; c < k; ++c) y2[i] += EV[(size_t)c * k + first + 1] * Q[c][i];
      }
    }
    if (res <= o.tol * rho) {
      converged = 1;
      break;
    }
    if (keep == 0 || breakdown || k < 2) {
      Y.clear();
      q = y;
      continue;
    }
    // thick restart: keep the smallest Ritz pairs above the threshold
    const int nkeep = std::min(std::min(keep, k - 1), k - first);
    std::vector<Vec> Ynew;
    Ynew.push_back(y);
    for (int c = 1; c < nkeep; ++c) {
      Vec yc(n, 0.0);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
      for (int64_t i = 0; i < n; ++i)
        for (int r = 0; r < k; ++r) yc[i] += EV[(size_t)r * k + first + c] * Q[r][i];
      Ynew.push_back(yc);
    }
    th_keep.assign(nkeep, 0.0);
    s_keep.assign(nkeep, 0.0);
    for (int c = 0; c < nkeep; ++c) {
      th_keep[c] = ev[first + c];
      s_keep[c] = last_b * EV[(size_t)(k - 1) * k + first + c];
    }
    Y.swap(Ynew);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
    for (int64_t i = 0; i < n; ++i) q[i] = w[i] / last_b;
  }
  info.theta = theta;
  info.residual = res;
  info.converged = converged;
  lambda = rayleigh(g, y, info.matvecs);
  canonical_sign(y, gid);
  return converged ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Block Lanczos for the Fiedler pair (Sec. 9: a block iteration of two
// vectors orthogonalised together at every step finds both vectors of an
// exactly degenerate pair, where a one-vector iteration finds only the
// combination its start vector holds).  The steps, in the order taken:
//  * start block: column 0 the usual start (random, or warm), column 1 the
//    random start of seed ^ ORC_SECOND_SEED; ones component removed; Cholesky
//    QR twice (below);
//  * block step j: W = L X_j; two classical Gram-Schmidt passes of both
//    columns against [u0, Q]; the projected matrix T = Q^T L Q takes the two
//    passes' summed coefficients as the columns of X_j (rows of the vectors
//    before it and of X_j itself, the 2 x 2 block on the diagonal
//    symmetrised); Cholesky QR twice of the remainder gives X_{j+1};
//  * after m/2 blocks (or when both columns of a remainder vanish): the
//    eigenpairs of T by cyclic Jacobi; the two smallest give the Ritz pairs
//    (theta1, y1), (theta2, y2), each tested by ||L y - theta y|| <= tol theta;
//  * restart: explicit from [y1, y2] (keep = 0), or thick (keep > 0, even):
//    the keep smallest Ritz vectors head the next cycle's basis, where T is
//    diag(theta), and the cycle continues from the last remainder block.
// Readings (the paper gives no algorithmic detail): T from the computed
// coefficients rather than an assumed block-tridiagonal form (the same in
// exact arithmetic; it also gives the couplings of the kept vectors);
// Cholesky QR run twice, the second on the nearly orthonormal first result.
// Deflation: a column whose part orthogonal to the column before it is at
// most kBlockDeflRel of its norm, or below kBlockDeflAbs times the largest
// ||L x|| seen, becomes a zero column; it stays zero in later blocks (the
// block continues as a one-vector Lanczos) and its diagonal entry of T is
// set above every eigenvalue of T, so that it never enters the pair.
// A pair within sweep_gap (when fiedler_sweep > 0) is rotated within its
// plane so that y1 is the normalised projection of the random start of seed
// on it: the pair's plane is well defined, a basis of it (for an exactly
// degenerate pair) is not.
// ---------------------------------------------------------------------------
constexpr double kBlockDeflRel = 1e-7;
constexpr double kBlockDeflAbs = 1e-10;

struct BlockQR {
  double r00 = 0.0, r01 = 0.0, r11 = 0.0;
  bool z0 = false, z1 = false;  // dropped (zero) columns
};

// [w0, w1] = [x0, x1] R by Cholesky QR of the Gram matrix (in place).
BlockQR block_cholqr(Vec &w0, Vec &w1, double thr_abs) {
  BlockQR r;
  const double g00 = dot(w0, w0), g01 = dot(w0, w1), g11 = dot(w1, w1);
  r.r00 = std::sqrt(g00);
  r.z0 = !(r.r00 > thr_abs);
  if (r.z0) {
    r.r00 = 0.0;
    r.r01 = 0.0;
  } else {
    r.r01 = g01 / r.r00;
  }
  r.r11 = std::sqrt(std::max(g11 - r.r01 * r.r01, 0.0));
  r.z1 = !(r.r11 > std::max(thr_abs, kBlockDeflRel * std::sqrt(g11)));
  if (r.z1) r.r11 = 0.0;
  const int64_t n = (int64_t)w0.size();
  for (int64_t i = 0; i < n; ++i) {
    const double x0 = r.z0 ? 0.0 : w0[i] / r.r00;
    const double x1 = r.z1 ? 0.0 : (w1[i] - r.r01 * x0) / r.r11;
    w0[i] = x0;
    w1[i] = x1;
  }
  return r;
}

// Both passes; the second keeps the first one's dropped columns dropped.
void block_cholqr2(Vec &w0, Vec &w1, double thr_abs, bool &z0, bool &z1) {
  const BlockQR a = block_cholqr(w0, w1, thr_abs);
  const BlockQR b = block_cholqr(w0, w1, 0.5);
  z0 = a.z0 || b.z0;
  z1 = a.z1 || b.z1;
}

int block_fiedler(const Graph &g, const std::vector<int64_t> &gid, const orc_opts &o, Vec &y,
                  double &lambda, orc_info &info, SecondPair &pair,
                  const WarmMap *warm = nullptr) {
  const int64_t n = g.n;
  const double u0 = 1.0 / std::sqrt((double)n);
  const int nb = std::max(2, o.lanczos_m) / 2;  // blocks per cycle
  const int keep = std::max(0, o.lanczos_keep);
  Vec x0(n), x1(n);
  double raw = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    x0[i] = start_value(o.seed, gid[i]);
    if (warm) {
      auto it = warm->find(gid[i]);
      if (it != warm->end()) x0[i] = it->second + kWarmNoise * x0[i];
    }
    x1[i] = start_value(o.seed ^ ORC_SECOND_SEED, gid[i]);
  }
  raw = std::sqrt(std::max(dot(x0, x0), dot(x1, x1)));
  deflate_ones(x0);
  deflate_ones(x1);
  bool z0 = false, z1 = false;
  block_cholqr2(x0, x1, kBlockDeflAbs * raw, z0, z1);
  std::vector<Vec> Q;          // basis of the cycle
  std::vector<char> zq;        // zero (dropped) columns of Q
  Vec tkeep;                   // Ritz values of the kept vectors at its head
  double tnorm = 0.0;
  int converged = 0;
  double th1 = 0.0, th2 = 0.0, res1 = 0.0;
  bool has2 = false;
  Vec y1(n, 0.0), y2(n, 0.0);
  for (int cycle = 0; cycle <= o.max_restarts; ++cycle) {
    const int nk = (int)Q.size();
    const int mv = nk + 2 * (nb - nk / 2);     // basis size of a full cycle
    Vec T((size_t)mv * mv, 0.0);
    for (int i = 0; i < nk; ++i) T[(size_t)i * mv + i] = tkeep[i];
    Q.push_back(x0);
    Q.push_back(x1);
    zq.push_back(z0);
    zq.push_back(z1);
    bool breakdown = false;
    for (int jb = nk / 2; jb < nb; ++jb) {
      const int a = 2 * jb;  // first column of X_j in Q
      Vec w0(n), w1(n);
      apply_laplacian(g, Q[a], w0);
      apply_laplacian(g, Q[a + 1], w1);
      info.matvecs += 2;
      tnorm = std::max(tnorm, std::max(norm2(w0), norm2(w1)));
      const int nq = a + 2;
      Vec hs((size_t)nq * 2, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        for (int c = 0; c < 2; ++c) {
          Vec &w = c ? w1 : w0;
          const double *pw = w.data();
          const double h0 = fixed_sum(n, [=](int64_t i) { return u0 * pw[i]; });
          std::vector<double> h(nq);
          for (int k = 0; k < nq; ++k) h[k] = dot(Q[k], w);
          for (int64_t i = 0; i < n; ++i) {
            double s = h0 * u0;
            for (int k = 0; k < nq; ++k) s += h[k] * Q[k][i];
            w[i] -= s;
          }
          for (int k = 0; k < nq; ++k) hs[(size_t)k * 2 + c] += h[k];
        }
      }
      for (int k = 0; k < a; ++k)
        for (int c = 0; c < 2; ++c)
          T[(size_t)k * mv + a + c] = T[(size_t)(a + c) * mv + k] = hs[(size_t)k * 2 + c];
      T[(size_t)a * mv + a] = hs[(size_t)a * 2 + 0];
      T[(size_t)(a + 1) * mv + a + 1] = hs[(size_t)(a + 1) * 2 + 1];
      T[(size_t)a * mv + a + 1] = T[(size_t)(a + 1) * mv + a] =
          0.5 * (hs[(size_t)a * 2 + 1] + hs[(size_t)(a + 1) * 2 + 0]);
      // the remainder block: the next X (or, after the last block, the
      // continuation of a thick restart)
      block_cholqr2(w0, w1, kBlockDeflAbs * tnorm, z0, z1);
      x0.swap(w0);
      x1.swap(w1);
      if (z0 && z1) {
        breakdown = true;
        break;
      }
      if (jb + 1 < nb) {
        Q.push_back(x0);
        Q.push_back(x1);
        zq.push_back(z0);
        zq.push_back(z1);
      }
    }
    // Ritz pairs of T (its leading k x k part)
    const int k = (int)Q.size();
    double big = 0.0;
    for (int r = 0; r < k; ++r) {
      if (zq[r]) continue;
      double rs = 0.0;
      for (int c = 0; c < k; ++c) rs += std::fabs(T[(size_t)r * mv + c]);
      big = std::max(big, rs);
    }
    big = 1.0 + 2.0 * big;
    Vec Tk((size_t)k * k);
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) Tk[(size_t)r * k + c] = T[(size_t)r * mv + c];
    for (int r = 0; r < k; ++r)
      if (zq[r]) Tk[(size_t)r * k + r] = big;
    Vec ev, EV;
    jacobi_eigen(k, Tk, ev, EV);
    const int nn = std::max(2, keep);
    std::vector<Vec> R(nn, Vec(n, 0.0));
    for (int c = 0; c < nn && c < k; ++c)
      for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int r = 0; r < k; ++r) s += EV[(size_t)r * k + c] * Q[r][i];
        R[c][i] = s;
      }
    th1 = ev[0];
    th2 = ev[1];
    has2 = ev[1] < big;
    y1 = R[0];
    y2 = R[1];
    res1 = residual_norm(g, y1, th1, info.matvecs);
    const double res2 = has2 ? residual_norm(g, y2, th2, info.matvecs) : 0.0;
    info.cycles = cycle + 1;
    if (res1 <= o.tol * th1 && (!has2 || res2 <= o.tol * th2)) {
      converged = 1;
      break;
    }
    if (cycle == o.max_restarts) break;
    if (keep == 0 || breakdown) {
      Q.clear();
      zq.clear();
      tkeep.clear();
      x0 = y1;
      x1 = y2;
      deflate_ones(x0);
      deflate_ones(x1);
      block_cholqr2(x0, x1, kBlockDeflAbs, z0, z1);
      continue;
    }
    // thick restart: x0, x1 hold the last remainder block
    Q.assign(R.begin(), R.begin() + keep);
    zq.assign(keep, 0);
    tkeep.assign(ev.begin(), ev.begin() + keep);
    for (int c = 0; c < keep; ++c) zq[c] = !(ev[c] < big);
  }
  if (o.fiedler_sweep > 0 && has2 && th2 - th1 <= o.sweep_gap * th1) {
    double c1 = 0.0, c2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double s = start_value(o.seed, gid[i]);
      c1 += s * y1[i];
      c2 += s * y2[i];
    }
    const double cn = std::sqrt(c1 * c1 + c2 * c2);
    if (cn > 0.0)
      for (int64_t i = 0; i < n; ++i) {
        const double a1 = y1[i], a2 = y2[i];
        y1[i] = (c1 * a1 + c2 * a2) / cn;
        y2[i] = (c1 * a2 - c2 * a1) / cn;
      }
  }
  normalize(y1);
  y = y1;
  info.theta = th1;
  info.residual = res1;
  info.converged = converged;
  lambda = rayleigh(g, y, info.matvecs);
  canonical_sign(y, gid);
  pair.ok = has2;
  pair.theta1 = th1;
  pair.theta2 = th2;
  pair.y2 = y2;
  return converged ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Aggregation multigrid preconditioner for the inverse-iteration solves
// (Sec. 7, Alg. 3).  Every level is the Laplacian of a graph with integer
// weights; the next level collapses pairs of rows (piecewise-constant
// prolongation J, Galerkin product J^T L J, which is again a graph
// Laplacian: the weight between two aggregates is the sum of the weights of
// the edges between their members, and edges inside an aggregate vanish).
//
// Readings (the paper pairs elements by an RCB ordering, which needs
// coordinates the partitioner is not given):
//  * pairs come from a handshake matching: in each of kMatchRounds rounds
//    every unmatched row proposes to its unmatched neighbour of largest
//    (weight, pair hash), ties to the smaller global id; two rows that
//    propose to each other are matched.  The pair hash is the splitmix64
//    output for counter max(gid) of the stream started at min(gid), so both
//    ends of an edge rank it alike.  Unmatched rows stay single;
//  * a coarse row is numbered by its first member (fine order) and carries
//    the smaller global id of its members;
//  * coarsening stops when the next level would keep more than 90% of the
//    rows, when a pair's two rows have more than kAmgCandCap entries
//    together, or after kAmgMaxLevels levels;
//  * V-cycle smoothing is damped Jacobi with weight sigma; Alg. 3 as printed
//    subtracts L u from an already updated residual after the coarse
//    correction; here every post-smoothing step takes the true residual
//    f - L u.  The coarsest level only runs the pre-smoothing steps.
// ---------------------------------------------------------------------------
constexpr int kMatchRounds = 4;
constexpr int kAmgMaxLevels = 40;
constexpr int kAmgCandCap = 1024;

struct AmgGraph {
  int64_t n = 0;
  std::vector<std::vector<std::pair<int64_t, int64_t>>> adj;  // (neighbour, weight), ascending
  std::vector<int64_t> gid;
};

struct AmgLevel {
  AmgGraph g;
  std::vector<int64_t> agg;  // row -> row of the next level (empty on the coarsest level)
  Vec dinv;                  // 1 / L_ii (0 for an isolated row)
};

uint32_t pair_priority(int64_t ga, int64_t gb) {
  const uint64_t lo = (uint64_t)std::min(ga, gb), hi = (uint64_t)std::max(ga, gb);
  return (uint32_t)(splitmix64_at(lo, hi) >> 32);
}

// Handshake matching; mate[i] = partner, or i for a single row.
std::vector<int64_t> handshake_matching(const AmgGraph &g) {
  std::vector<int64_t> mate(g.n, -1), prop(g.n);
  for (int round = 0; round < kMatchRounds; ++round) {
    for (int64_t i = 0; i < g.n; ++i) {
      prop[i] = -1;
      if (mate[i] >= 0) continue;
      int64_t bw = -1;
      uint32_t bh = 0;
      for (auto &nw : g.adj[i]) {
        const int64_t j = nw.first;
        if (mate[j] >= 0) continue;
        const uint32_t h = pair_priority(g.gid[i], g.gid[j]);
        const bool better = prop[i] < 0 || nw.second > bw || (nw.second == bw && h > bh) ||
                            (nw.second == bw && h == bh && g.gid[j] < g.gid[prop[i]]);
        if (better) {
          prop[i] = j;
          bw = nw.second;
          bh = h;
        }
      }
    }
    std::vector<int64_t> matched;
    for (int64_t i = 0; i < g.n; ++i)
      if (mate[i] < 0 && prop[i] >= 0 && prop[prop[i]] == i) matched.push_back(i);
    for (int64_t i : matched) mate[i] = prop[i];
  }
  for (int64_t i = 0; i < g.n; ++i)
    if (mate[i] < 0) mate[i] = i;
  return mate;
}

Vec diag_inverse(const AmgGraph &g) {
  Vec d(g.n, 0.0);
  for (int64_t i = 0; i < g.n; ++i) {
    int64_t deg = 0;
    for (auto &nw : g.adj[i]) deg += nw.second;
    d[i] = deg > 0 ? 1.0 / (double)deg : 0.0;
  }
  return d;
}

// Coarse graph of the matching, or false if coarsening stops here.
bool coarsen(const AmgGraph &g, std::vector<int64_t> &agg, AmgGraph &c) {
  std::vector<int64_t> mate = handshake_matching(g);
  int64_t nc = 0;
  for (int64_t i = 0; i < g.n; ++i) {
    if (mate[i] < i) continue;  // the pair is numbered by its first member
    if ((int64_t)(g.adj[i].size() + (mate[i] != i ? g.adj[mate[i]].size() : 0)) > kAmgCandCap)
      return false;
    ++nc;
  }
  if (10 * nc > 9 * g.n) return false;
  agg.assign(g.n, -1);
  c.n = nc;
  c.adj.assign(nc, {});
  c.gid.assign(nc, 0);
  int64_t k = 0;
  for (int64_t i = 0; i < g.n; ++i)
    if (mate[i] >= i) {
      agg[i] = agg[mate[i]] = k;
      c.gid[k] = std::min(g.gid[i], g.gid[mate[i]]);
      ++k;
    }
  for (int64_t I = 0; I < nc; ++I) c.adj[I].clear();
  std::vector<std::map<int64_t, int64_t>> rows(nc);
  for (int64_t i = 0; i < g.n; ++i)
    for (auto &nw : g.adj[i])
      if (agg[nw.first] != agg[i]) rows[agg[i]][agg[nw.first]] += nw.second;
  for (int64_t I = 0; I < nc; ++I)
    for (auto &kv : rows[I]) c.adj[I].push_back(kv);
  return true;
}

std::vector<AmgLevel> amg_setup(const Graph &g0, const std::vector<int64_t> &gid) {
  std::vector<AmgLevel> lv(1);
  lv[0].g.n = g0.n;
  lv[0].g.gid = gid;
  lv[0].g.adj.resize(g0.n);
  for (int64_t i = 0; i < g0.n; ++i)
    for (auto &nw : g0.adj[i]) lv[0].g.adj[i].push_back({nw.first, nw.second});
  while ((int)lv.size() < kAmgMaxLevels) {
    AmgLevel next;
    if (!coarsen(lv.back().g, lv.back().agg, next.g)) {
      lv.back().agg.clear();
      break;
    }
    lv.push_back(std::move(next));
  }
  for (auto &l : lv) l.dinv = diag_inverse(l.g);
  return lv;
}

void amg_apply_laplacian(const AmgGraph &g, const Vec &x, Vec &y) {
  for (int64_t i = 0; i < g.n; ++i) {
    double s = 0.0;
    for (auto &nw : g.adj[i]) s += (double)nw.second * (x[i] - x[nw.first]);
    y[i] = s;
  }
}

// u = M_l f: one V-cycle from level l (Alg. 3 with the readings above).
void vcycle(const std::vector<AmgLevel> &lv, size_t l, const Vec &f, double sigma, int nsmooth,
            Vec &u) {
  const AmgLevel &L = lv[l];
  const int64_t n = L.g.n;
  Vec r(n), lu(n);
  u.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) u[i] = sigma * L.dinv[i] * f[i];
  auto residual = [&]() {
    amg_apply_laplacian(L.g, u, lu);
    for (int64_t i = 0; i < n; ++i) r[i] = f[i] - lu[i];
  };
  residual();
  for (int s = 0; s < nsmooth; ++s) {
    for (int64_t i = 0; i < n; ++i) u[i] += sigma * L.dinv[i] * r[i];
    residual();
  }
  if (L.agg.empty()) return;  // coarsest level: smoothing only
  Vec fc(lv[l + 1].g.n, 0.0), ec;
  for (int64_t i = 0; i < n; ++i) fc[L.agg[i]] += r[i];
  vcycle(lv, l + 1, fc, sigma, nsmooth, ec);
  for (int64_t i = 0; i < n; ++i) u[i] += ec[L.agg[i]];
  for (int s = 0; s < nsmooth; ++s) {
    residual();
    for (int64_t i = 0; i < n; ++i) u[i] += sigma * L.dinv[i] * r[i];
  }
}

// Conjugate gradients for L x = b with b orthogonal to the ones vector
// (Sec. 7): x0 = 0, first direction r0 (not preconditioned), then the
// preconditioned residual z = M r (identity, or one V-cycle with the ones
// component removed) and the flexible (Polak-Ribiere) beta
// z_new^T (r_new - r_old) / z_old^T r_old; optional L-orthogonalisation of
// every new direction against the kept ones ("full projection").
// Returns iterations.
// If dirs is given, every search direction p is appended to it before its
// step (test hook: the directions of one solve).
int cg_solve(const Graph &g, const Vec &b, const orc_opts &o, const std::vector<AmgLevel> *amg,
             Vec &x, int64_t &matvecs, std::vector<Vec> *dirs = nullptr) {
  const int64_t n = g.n;
  x.assign(n, 0.0);
  Vec r = b, p, lp(n), z;
  deflate_ones(r);
  p = r;
  z = r;
  double rz = dot(r, z);
  double bnorm = norm2(b);
  std::vector<Vec> P, LP;
  std::vector<double> pLp;
  int it = 0;
  if (norm2(r) <= o.cg_tol * bnorm) return 0;
  for (it = 1; it <= o.cg_max_iter; ++it) {
    if (dirs) dirs->push_back(p);
    apply_laplacian(g, p, lp);
    ++matvecs;
    double plp = dot(p, lp);
    double alpha = rz / plp;
    Vec rn(n);
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
    for (int64_t i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      rn[i] = r[i] - alpha * lp[i];
    }
    deflate_ones(rn);
    if (norm2(rn) <= o.cg_tol * bnorm) break;
    Vec zn;
    if (amg) {
      vcycle(*amg, 0, rn, o.amg_sigma, o.amg_smooth, zn);
      deflate_ones(zn);
    } else {
      zn = rn;
    }
    const double *pz = zn.data(), *prn = rn.data(), *pr = r.data();
    const double diff = fixed_sum(n, [=](int64_t i) { return pz[i] * (prn[i] - pr[i]); });
    double beta = diff / rz;
    if (o.cg_full_projection > 0) {
      P.push_back(p);
      LP.push_back(lp);
      pLp.push_back(plp);
      if ((int)P.size() > o.cg_full_projection) {
        P.erase(P.begin());
        LP.erase(LP.begin());
        pLp.erase(pLp.begin());
      }
    }
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
    for (int64_t i = 0; i < n; ++i) p[i] = zn[i] + beta * p[i];
    for (size_t k = 0; k < P.size(); ++k) {
      double c = dot(LP[k], p) / pLp[k];
      const double *pk = P[k].data();
      double *pp = p.data();
#pragma omp parallel for schedule(static) if (n >= kThreadMin)
      for (int64_t i = 0; i < n; ++i) pp[i] -= c * pk[i];
    }
    r = rn;
    z = zn;
    rz = dot(r, z);
  }
  return std::min(it, o.cg_max_iter);
}

// Inverse iteration (Sec. 7, Alg. 2).
int inverse_fiedler(const Graph &g, const std::vector<int64_t> &gid, const orc_opts &o, Vec &y,
                    double &lambda, orc_info &info) {
  const int64_t n = g.n;
  Vec b(n), x;
  for (int64_t i = 0; i < n; ++i) b[i] = start_value(o.seed, gid[i]);
  int converged = 0;
  double rho = 0.0, res = 0.0;
  std::vector<AmgLevel> amg;
  if (o.inv_precond == ORC_PRECOND_AMG) amg = amg_setup(g, gid);
  info.amg_levels = (int32_t)amg.size();
  for (int outer = 0; outer < o.inv_max_outer; ++outer) {
    deflate_ones(b);
    normalize(b);
    int its = cg_solve(g, b, o, amg.empty() ? nullptr : &amg, x, info.matvecs);
    info.cg_iters += its;
    b = x;
    info.cycles = outer + 1;
    // eigen-residual of the new iterate
    Vec yy = b;
    deflate_ones(yy);
    normalize(yy);
    rho = rayleigh(g, yy, info.matvecs);
    res = residual_norm(g, yy, rho, info.matvecs);
    if (its <= 1 || res <= o.tol * rho) {
      converged = 1;
      break;
    }
  }
  deflate_ones(b);
  normalize(b);
  y = b;
  info.theta = rho;
  info.residual = res;
  info.converged = converged;
  lambda = rayleigh(g, y, info.matvecs);
  canonical_sign(y, gid);
  return converged ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Components, split rule, recursion (Sec. 4, Alg. 1)
// ---------------------------------------------------------------------------

// Component of every vertex, numbered in order of each component's smallest
// global id.
int components(const Graph &g, const std::vector<int64_t> &gid, std::vector<int32_t> &comp) {
  comp.assign(g.n, -1);
  int nc = 0;
  std::vector<int32_t> stack;
  for (int64_t s = 0; s < g.n; ++s) {
    if (comp[s] >= 0) continue;
    comp[s] = nc;
    stack.push_back((int32_t)s);
    while (!stack.empty()) {
      int32_t u = stack.back();
      stack.pop_back();
      for (auto &nw : g.adj[u])
        if (comp[nw.first] < 0) {
          comp[nw.first] = nc;
          stack.push_back(nw.first);
        }
    }
    ++nc;
  }
  std::vector<int64_t> mingid(nc, INT64_MAX);
  for (int64_t i = 0; i < g.n; ++i) mingid[comp[i]] = std::min(mingid[comp[i]], gid[i]);
  std::vector<int32_t> order(nc), rank(nc);
  for (int c = 0; c < nc; ++c) order[c] = c;
  std::sort(order.begin(), order.end(),
            [&](int32_t a, int32_t b) { return mingid[a] < mingid[b]; });
  for (int c = 0; c < nc; ++c) rank[order[c]] = c;
  for (auto &c : comp) c = rank[c];
  return nc;
}

// Induced subgraph on the sorted local index list `keep`.
Graph induced(const Graph &g, const std::vector<int64_t> &keep) {
  std::unordered_map<int64_t, int32_t> local;
  for (size_t i = 0; i < keep.size(); ++i) local[keep[i]] = (int32_t)i;
  Graph s;
  s.n = (int64_t)keep.size();
  s.adj.resize(s.n);
  for (size_t i = 0; i < keep.size(); ++i)
    for (auto &nw : g.adj[keep[i]]) {
      auto it = local.find(nw.first);
      if (it != local.end()) s.adj[i].push_back({it->second, nw.second});
    }
  for (auto &a : s.adj) std::sort(a.begin(), a.end());
  return s;
}

// Total order on doubles used for the split key: -0.0 before +0.0.
uint64_t ordered_bits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, 8);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ULL);
}

struct KeyLess {
  const Vec &y;
  const std::vector<int64_t> &gid;
  bool operator()(int64_t a, int64_t b) const {
    uint64_t ka = ordered_bits(y[a]), kb = ordered_bits(y[b]);
    if (ka != kb) return ka < kb;
    return gid[a] < gid[b];
  }
};

// side[i] = 0 for the n_low smallest keys (y_i, gid_i).
void split_by_keys(const Vec &y, const std::vector<int64_t> &gid, int64_t n_low,
                   std::vector<uint8_t> &side) {
  std::vector<int64_t> order(y.size());
  for (size_t i = 0; i < y.size(); ++i) order[i] = (int64_t)i;
  std::sort(order.begin(), order.end(), KeyLess{y, gid});
  side.assign(y.size(), 1);
  for (int64_t r = 0; r < n_low; ++r) side[order[r]] = 0;
}

struct SolveResult {
  int status = 0;         // 0 ok, 1 not converged, 2 disconnected
  double lambda = 0.0;
};

// Weight of the edges between the two sides of a bisection.
int64_t bisection_cut(const Graph &g, const std::vector<uint8_t> &side) {
  int64_t cut = 0;
  for (int64_t i = 0; i < g.n; ++i)
    for (auto &nw : g.adj[i])
      if (nw.first > i && side[i] != side[nw.first]) cut += nw.second;
  return cut;
}

// Sweep over the Fiedler pair (the paper's suggestion for a degenerate pair,
// Sec. 9): when the second Ritz value is within sweep_gap (relative) of the
// first, y1 and the second Ritz vector orthonormalised against u0 and y1,
// each with the canonical sign, are combined as cos(a) y1 + sin(a) y2 for
// a = k pi / S, k = 0..S-1; every combination (canonical sign) is split by
// the usual rule and the one of smallest cut replaces y (ties: smallest k).
bool sweep_pair(const Graph &g, const std::vector<int64_t> &gid, int64_t n_low, const orc_opts &o,
                const SecondPair &sp, Vec &y, orc_info &info, double min_perp = 1e-6) {
  if (!(sp.theta2 - sp.theta1 <= o.sweep_gap * sp.theta1)) return false;
  const int64_t n = g.n;
  Vec y2 = sp.y2;
  deflate_ones(y2);
  const double b = dot(y, y2);
  for (int64_t i = 0; i < n; ++i) y2[i] -= b * y[i];
  const double nn = norm2(y2);
  if (!(nn > min_perp)) return false;
  for (double &v : y2) v /= nn;
  canonical_sign(y2, gid);
  info.sweeps += 1;
  int64_t best_cut = -1;
  int best = 0;
  Vec best_y;
  for (int k = 0; k < o.fiedler_sweep; ++k) {
    const double a = M_PI * (double)k / (double)o.fiedler_sweep;
    const double c = std::cos(a), sn = std::sin(a);
    Vec yk(n);
    for (int64_t i = 0; i < n; ++i) yk[i] = c * y[i] + sn * y2[i];
    canonical_sign(yk, gid);
    std::vector<uint8_t> side;
    split_by_keys(yk, gid, n_low, side);
    const int64_t cut = bisection_cut(g, side);
    if (best_cut < 0 || cut < best_cut) {
      best_cut = cut;
      best = k;
      best_y = yk;
    }
  }
  if (best != 0) info.sweep_moved += 1;
  y = best_y;
  return true;
}

// One bisection of graph g (vertices in ascending gid order) into a low side
// of n_low vertices and a high side.  y receives the vector used (zero
// outside the component that was cut).  Returns the status of the solve.
int bisect(const Graph &g, const std::vector<int64_t> &gid, int64_t n_low, const orc_opts &o,
           std::vector<uint8_t> &side, Vec &y, double &lambda, orc_info &info,
           WarmMap *warm = nullptr) {
  std::vector<int32_t> comp;
  int nc = components(g, gid, comp);
  info.ncomp = nc;
  std::vector<int64_t> size(nc, 0);
  for (int32_t c : comp) size[c] += 1;
  // components are numbered in order of their smallest global id
  int64_t before = 0;
  int strad = -1;
  int64_t strad_before = 0;
  for (int c = 0; c < nc; ++c) {
    if (before < n_low && n_low < before + size[c]) {
      strad = c;
      strad_before = before;
    }
    before += size[c];
  }
  side.assign(g.n, 1);
  y.assign(g.n, 0.0);
  lambda = 0.0;
  std::vector<int64_t> prefix(nc, 0);
  for (int c = 1; c < nc; ++c) prefix[c] = prefix[c - 1] + size[c - 1];
  for (int64_t i = 0; i < g.n; ++i) {
    int c = comp[i];
    if (prefix[c] + size[c] <= n_low) side[i] = 0;
  }
  int status = (nc > 1) ? 2 : 0;
  if (strad < 0) return status;
  std::vector<int64_t> members;
  for (int64_t i = 0; i < g.n; ++i)
    if (comp[i] == strad) members.push_back(i);
  Graph sub = (nc > 1) ? induced(g, members) : g;
  std::vector<int64_t> sub_gid(members.size());
  for (size_t i = 0; i < members.size(); ++i) sub_gid[i] = gid[members[i]];
  Vec ys;
  int st;
  SecondPair second;
  if (o.method == ORC_INVERSE_CG) {
    st = inverse_fiedler(sub, sub_gid, o, ys, lambda, info);
  } else if (o.method == ORC_BLOCK) {
    st = block_fiedler(sub, sub_gid, o, ys, lambda, info, second, warm);
  } else {
    st = lanczos_fiedler(sub, sub_gid, o, ys, lambda, info,
                         (o.fiedler_sweep > 0 || warm) ? &second : nullptr, warm);
    // ORC_AUTO (Sec. 7: inverse iteration where Lanczos does not converge):
    // a fresh inverse-iteration solve from the random start replaces the
    // result; the second Ritz vector of the Lanczos run is still handed on
    if (o.method == ORC_AUTO && st == 1) {
      info.fallbacks += 1;
      st = inverse_fiedler(sub, sub_gid, o, ys, lambda, info);
    }
  }
  if (st < 0) return st;
  if (warm && second.ok) {
    // values for the children: y2 at unit root-mean-square on the component
    double nn = 0.0;
    for (double v : second.y2) nn += v * v;
    const double scale = std::sqrt((double)sub_gid.size()) / std::sqrt(nn);
    for (size_t i = 0; i < sub_gid.size(); ++i) (*warm)[sub_gid[i]] = second.y2[i] * scale;
  }
  std::vector<uint8_t> sub_side;
  if (o.second_solve && o.fiedler_sweep > 0 && o.method != ORC_INVERSE_CG &&
      o.method != ORC_BLOCK) {
    // the pair from two solves: Lanczos again from another random start
    // (no warm start); a second vector within sweep_gap of the first and at
    // least 0.1 away from its direction is swept with it, a vector the
    // solve brought back to y1 is not
    orc_opts o2 = o;
    o2.seed = o.seed ^ ORC_SECOND_SEED;
    orc_info i2{};
    SecondPair two;
    double lam2 = 0.0;
    const int s2 = lanczos_fiedler(sub, sub_gid, o2, two.y2, lam2, i2);
    if (s2 < 0) return s2;
    info.matvecs += i2.matvecs;
    two.ok = true;
    two.theta1 = lambda;
    two.theta2 = lam2;
    // a second solve that did not give a pair to sweep leaves the thick
    // restart's own pair (its Ritz values, its second Ritz vector)
    if (!sweep_pair(sub, sub_gid, n_low - strad_before, o, two, ys, info, 0.1) && second.ok)
      sweep_pair(sub, sub_gid, n_low - strad_before, o, second, ys, info);
  } else if (second.ok && o.fiedler_sweep > 0) {
    sweep_pair(sub, sub_gid, n_low - strad_before, o, second, ys, info);
  }
  split_by_keys(ys, sub_gid, n_low - strad_before, sub_side);
  for (size_t i = 0; i < members.size(); ++i) {
    side[members[i]] = sub_side[i];
    y[members[i]] = ys[i];
  }
  if (status == 0 && st == 1) status = 1;
  return status;
}

void to_graph(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
              Graph &g) {
  g.n = n;
  g.adj.assign(n, {});
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) g.adj[i].push_back({col[p], weight[p]});
}

bool valid_mesh(int64_t nelem, int32_t nv, const int64_t *ids) {
  if (nelem < 1 || nv < 1 || !ids) return false;
  for (int64_t i = 0; i < nelem * nv; ++i)
    if (ids[i] < 0) return false;
  return true;
}

// Recursion of Alg. 1 on the vertex list `elems` (ascending global ids),
// parts [p0, p0 + np).  The first call (root) reads the start values of
// bfs_start from `warm`; the others read it only with warm_start.
int rsb_recurse(const Graph &g, const std::vector<int64_t> &elems, int32_t p0, int32_t np,
                const orc_opts &o, int32_t *part, orc_info &info, int &worst, WarmMap &warm,
                bool root = false) {
  if (np == 1) {
    for (int64_t e : elems) part[e] = p0;
    return 0;
  }
  Graph sub = induced(g, elems);
  int32_t pl = np / 2;
  int64_t n_low = (int64_t)((__int128)elems.size() * pl / np);
  std::vector<uint8_t> side;
  Vec y;
  double lam;
  orc_info li{};
  const bool read_warm = o.warm_start || (root && o.bfs_start);
  int st = bisect(sub, elems, n_low, o, side, y, lam, li, read_warm ? &warm : nullptr);
  if (st < 0) return st;
  worst = std::max(worst, st);
  info.matvecs += li.matvecs;
  info.cycles += li.cycles;
  info.cg_iters += li.cg_iters;
  info.sweeps += li.sweeps;
  info.sweep_moved += li.sweep_moved;
  info.fallbacks += li.fallbacks;
  std::vector<int64_t> lo, hi;
  for (size_t i = 0; i < elems.size(); ++i) (side[i] ? hi : lo).push_back(elems[i]);
  int r = rsb_recurse(g, lo, p0, pl, o, part, info, worst, warm);
  if (r < 0) return r;
  return rsb_recurse(g, hi, p0 + pl, np - pl, o, part, info, worst, warm);
}

// ---------------------------------------------------------------------------
// Locality order of the rows.  Not a step of the paper's method, which
// pre-sorts elements by recursive coordinate bisection before partitioning
// (that needs coordinates, which the input does not carry).  Classic
// Cuthill-McKee in its queue form: breadth-first search from a
// pseudo-peripheral row -- the row farthest from row 0, smallest index among
// the farthest -- where each row taken from the queue appends its unvisited
// neighbours in increasing index; rows the search never reaches follow in
// increasing index.  order[k] = old row placed at position k.
// ---------------------------------------------------------------------------
std::vector<int32_t> bfs_levels(const Graph &g, int64_t src) {
  std::vector<int32_t> dist(g.n, -1);
  std::vector<int64_t> queue{src};
  dist[src] = 0;
  for (size_t h = 0; h < queue.size(); ++h) {
    const int64_t i = queue[h];
    for (auto &e : g.adj[i])
      if (dist[e.first] < 0) {
        dist[e.first] = dist[i] + 1;
        queue.push_back(e.first);
      }
  }
  return dist;
}

// Start values of bfs_start (not in the paper, which leaves the start vector
// open): the number of edges from the pseudo-peripheral row (as for the
// locality order), centred and scaled to unit root-mean-square over the rows
// the search reaches (sums of the integer distances taken exactly).
void bfs_start_values(const Graph &g, const std::vector<int64_t> &gid, WarmMap &warm) {
  if (g.n < 2) return;
  const std::vector<int32_t> d0 = bfs_levels(g, 0);
  int64_t far = 0;
  for (int64_t i = 0; i < g.n; ++i)
    if (d0[i] > d0[far]) far = i;
  const std::vector<int32_t> d = bfs_levels(g, far);
  int64_t cnt = 0, s1 = 0, s2 = 0;
  for (int64_t i = 0; i < g.n; ++i)
    if (d[i] >= 0) {
      ++cnt;
      s1 += d[i];
      s2 += (int64_t)d[i] * d[i];
    }
  const double mean = (double)s1 / (double)cnt;
  const double var = (double)s2 / (double)cnt - mean * mean;
  if (cnt < 2 || !(var > 0.0)) return;
  const double sd = std::sqrt(var);
  for (int64_t i = 0; i < g.n; ++i)
    if (d[i] >= 0) warm[gid[i]] = ((double)d[i] - mean) / sd;
}

std::vector<int32_t> cuthill_mckee(Graph g) {
  for (auto &a : g.adj) std::sort(a.begin(), a.end());
  const std::vector<int32_t> d0 = bfs_levels(g, 0);
  int64_t far = 0;
  for (int64_t i = 0; i < g.n; ++i)
    if (d0[i] > d0[far]) far = i;
  std::vector<char> seen(g.n, 0);
  std::vector<int32_t> order{(int32_t)far};
  seen[far] = 1;
  for (size_t h = 0; h < order.size(); ++h)
    for (auto &e : g.adj[order[h]])
      if (!seen[e.first]) {
        seen[e.first] = 1;
        order.push_back(e.first);
      }
  for (int64_t i = 0; i < g.n; ++i)
    if (!seen[i]) order.push_back((int32_t)i);
  return order;
}

}  // namespace

extern "C" {

void orc_opts_default(orc_opts *o) {
  o->graph = ORC_GRAPH_WEIGHTED;
  o->method = ORC_LANCZOS;
  o->lanczos_m = 100;
  o->max_restarts = 50;
  o->tol = 1e-6;
  o->inv_max_outer = 50;
  o->cg_max_iter = 20000;
  o->cg_tol = 1e-8;
  o->cg_full_projection = 0;
  o->seed = 20261203ULL;
  o->lanczos_keep = 0;
  o->inv_precond = ORC_PRECOND_NONE;
  o->amg_smooth = 1;
  o->amg_sigma = 2.0 / 3.0;
  o->fiedler_sweep = 0;
  o->sweep_gap = 0.1;
  o->warm_start = 0;
  o->second_solve = 0;
  o->lanczos_s = 1;
  o->bfs_start = 0;
}

double orc_start_value(uint64_t seed, int64_t gid) { return start_value(seed, gid); }

int orc_dual_graph(int64_t nelem, int32_t nv, const int64_t *ids, int32_t graph, int64_t *row_ptr,
                   int32_t *col, int32_t *weight, int64_t *nnz_inout) {
  if (!valid_mesh(nelem, nv, ids) || !row_ptr || !nnz_inout) return -1;
  Graph g = build_dual_graph(nelem, nv, ids, graph);
  row_ptr[0] = 0;
  for (int64_t i = 0; i < nelem; ++i) row_ptr[i + 1] = row_ptr[i] + (int64_t)g.adj[i].size();
  int64_t nnz = row_ptr[nelem];
  if (!col) {
    *nnz_inout = nnz;
    return 0;
  }
  if (*nnz_inout < nnz) {
    *nnz_inout = nnz;
    return -4;
  }
  for (int64_t i = 0; i < nelem; ++i)
    for (size_t p = 0; p < g.adj[i].size(); ++p) {
      col[row_ptr[i] + p] = g.adj[i][p].first;
      if (weight) weight[row_ptr[i] + p] = g.adj[i][p].second;
    }
  *nnz_inout = nnz;
  return 0;
}

void orc_laplacian_apply(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *weight, const double *x, double *y) {
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  Vec xv(x, x + n), yv(n);
  apply_laplacian(g, xv, yv);
  std::copy(yv.begin(), yv.end(), y);
}

int orc_tridiag_smallest(int32_t k, const double *a, const double *b, double spurious_thr,
                         double *theta, double *t) {
  Vec tv;
  int r = tridiag_smallest(k, a, b, spurious_thr, theta, tv);
  if (r == 0) std::copy(tv.begin(), tv.end(), t);
  return r;
}

void orc_jacobi_eigen(int32_t k, const double *A, double *ev, double *V) {
  Vec a(A, A + (size_t)k * k), e, v;
  jacobi_eigen(k, a, e, v);
  std::copy(e.begin(), e.end(), ev);
  std::copy(v.begin(), v.end(), V);
}

int orc_fiedler_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                    const int64_t *gid, const orc_opts *o, double *y, double *lambda,
                    orc_info *info) {
  if (n < 2 || !row_ptr || !col || !weight || !gid || !o || !y || !lambda) return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  std::vector<int64_t> gv(gid, gid + n);
  std::vector<uint8_t> side;
  Vec yv;
  orc_info li{};
  int st = bisect(g, gv, n / 2, *o, side, yv, *lambda, li);
  if (info) *info = li;
  if (st < 0) return st;
  std::copy(yv.begin(), yv.end(), y);
  return st;
}

int orc_block_pair(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                   const int64_t *gid, const orc_opts *o, double *y1, double *y2, double *theta,
                   orc_info *info) {
  if (n < 2 || !row_ptr || !col || !weight || !gid || !o || !y1 || !y2 || !theta) return -1;
  if (o->lanczos_m < 4 || o->lanczos_m % 2 || o->lanczos_keep < 0 || o->lanczos_keep % 2 ||
      o->lanczos_keep > o->lanczos_m - 4)
    return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  std::vector<int64_t> gv(gid, gid + n);
  std::vector<int32_t> comp;
  if (components(g, gv, comp) != 1) return -2;
  Vec yv;
  double lambda = 0.0;
  orc_info li{};
  SecondPair pair;
  const int st = block_fiedler(g, gv, *o, yv, lambda, li, pair);
  if (info) *info = li;
  std::copy(yv.begin(), yv.end(), y1);
  for (int64_t i = 0; i < n; ++i) y2[i] = pair.y2[i];
  theta[0] = pair.theta1;
  theta[1] = pair.ok ? pair.theta2 : INFINITY;
  return st;
}

int orc_cg_solve(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                 const int64_t *gid, const orc_opts *o, const double *b, double *x,
                 int32_t max_dirs, double *dirs, int32_t *ndirs) {
  if (n < 2 || !row_ptr || !col || !weight || !gid || !o || !b || !x) return -1;
  if (max_dirs < 0 || (max_dirs > 0 && (!dirs || !ndirs))) return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  std::vector<int64_t> gv(gid, gid + n);
  std::vector<AmgLevel> amg;
  if (o->inv_precond == ORC_PRECOND_AMG) amg = amg_setup(g, gv);
  Vec bv(b, b + n), xv;
  std::vector<Vec> dv;
  int64_t matvecs = 0;
  const int its = cg_solve(g, bv, *o, amg.empty() ? nullptr : &amg, xv, matvecs,
                           max_dirs > 0 ? &dv : nullptr);
  std::copy(xv.begin(), xv.end(), x);
  if (max_dirs > 0) {
    const int32_t nd = (int32_t)std::min<size_t>(dv.size(), (size_t)max_dirs);
    for (int32_t k = 0; k < nd; ++k) std::copy(dv[k].begin(), dv[k].end(), dirs + (int64_t)k * n);
    *ndirs = nd;
  }
  return its;
}

int orc_set_threads(int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads >= 1) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

int orc_fiedler(int64_t nelem, int32_t nv, const int64_t *ids, const orc_opts *o, double *y,
                double *lambda, orc_info *info) {
  if (!valid_mesh(nelem, nv, ids) || nelem < 2 || !o || !y || !lambda) return -1;
  Graph g = build_dual_graph(nelem, nv, ids, o->graph);
  std::vector<int64_t> gv(nelem);
  for (int64_t i = 0; i < nelem; ++i) gv[i] = i;
  std::vector<uint8_t> side;
  Vec yv;
  orc_info li{};
  WarmMap warm;
  if (o->bfs_start) bfs_start_values(g, gv, warm);
  int st = bisect(g, gv, nelem / 2, *o, side, yv, *lambda, li, o->bfs_start ? &warm : nullptr);
  if (info) *info = li;
  if (st < 0) return st;
  std::copy(yv.begin(), yv.end(), y);
  return st;
}

int orc_split(int64_t n, const double *y, const int64_t *gid, int64_t n_low, uint8_t *side) {
  if (n < 0 || n_low < 0 || n_low > n || (n > 0 && (!y || !gid || !side))) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (std::isnan(y[i])) return -1;
  Vec yv(y, y + n);
  std::vector<int64_t> gv(gid, gid + n);
  std::vector<uint8_t> s;
  split_by_keys(yv, gv, n_low, s);
  std::copy(s.begin(), s.end(), side);
  return 0;
}

int orc_amg_level(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                  const int64_t *gid, int32_t level, int32_t *nlevels, int64_t *nrows,
                  int64_t *nnz, int64_t *row_ptr_out, int64_t *col_out, int64_t *weight_out,
                  int64_t *gid_out, int64_t *agg) {
  if (n < 1 || !row_ptr || !gid || !nlevels || !nrows || !nnz) return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  std::vector<int64_t> gv(gid, gid + n);
  std::vector<AmgLevel> lv = amg_setup(g, gv);
  *nlevels = (int32_t)lv.size();
  if (level < 0 || level >= (int32_t)lv.size()) return -1;
  const AmgLevel &L = lv[level];
  *nrows = L.g.n;
  int64_t k = 0;
  for (int64_t i = 0; i < L.g.n; ++i) k += (int64_t)L.g.adj[i].size();
  *nnz = k;
  if (row_ptr_out && col_out && weight_out) {
    k = 0;
    for (int64_t i = 0; i < L.g.n; ++i) {
      row_ptr_out[i] = k;
      for (auto &nw : L.g.adj[i]) {
        col_out[k] = nw.first;
        weight_out[k] = nw.second;
        ++k;
      }
    }
    row_ptr_out[L.g.n] = k;
  }
  if (gid_out)
    for (int64_t i = 0; i < L.g.n; ++i) gid_out[i] = L.g.gid[i];
  if (agg)
    for (int64_t i = 0; i < L.g.n; ++i) agg[i] = L.agg.empty() ? -1 : L.agg[i];
  return 0;
}

// Gather-scatter form of the weighted Laplacian (Sec. 5): each element's
// value is copied to its distinct vertices (P), the copies are summed per
// vertex (Q Q^T) and gathered back (P^T), so (A_w x)_e = sum over e's
// vertices v of u_v, u_v = sum of x over the elements containing v; with
// D = diag(A_w 1), L x = D x - A_w x.
int orc_gs_apply(int64_t nelem, int32_t nv, const int64_t *ids, const double *x, double *y) {
  if (!valid_mesh(nelem, nv, ids) || !x || !y) return -1;
  std::vector<std::vector<int64_t>> verts(nelem);
  std::map<int64_t, double> u, count;
  for (int64_t e = 0; e < nelem; ++e) {
    std::set<int64_t> d(ids + e * nv, ids + (e + 1) * nv);
    verts[e].assign(d.begin(), d.end());
    for (int64_t v : verts[e]) {
      u[v] += x[e];
      count[v] += 1.0;
    }
  }
  for (int64_t e = 0; e < nelem; ++e) {
    double ax = 0.0, diag = 0.0;
    for (int64_t v : verts[e]) {
      ax += u[v];
      diag += count[v];
    }
    y[e] = diag * x[e] - ax;
  }
  return 0;
}

int orc_locality_order(int64_t n, const int64_t *row_ptr, const int32_t *col,
                       const int32_t *weight, int32_t *order) {
  if (n < 1 || !row_ptr || !col || !weight || !order) return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  const std::vector<int32_t> o = cuthill_mckee(g);
  std::copy(o.begin(), o.end(), order);
  return 0;
}

int orc_bfs_start(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                  double *out) {
  if (n < 1 || !row_ptr || !col || !weight || !out) return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  std::vector<int64_t> gv(n);
  for (int64_t i = 0; i < n; ++i) gv[i] = i;
  WarmMap warm;
  bfs_start_values(g, gv, warm);
  for (int64_t i = 0; i < n; ++i) {
    auto it = warm.find(i);
    out[i] = it == warm.end() ? std::nan("") : it->second;
  }
  return 0;
}

int orc_amg_vcycle(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                   const int64_t *gid, double sigma, int32_t nsmooth, const double *f, double *u) {
  if (n < 1 || !row_ptr || !gid || !f || !u || nsmooth < 0) return -1;
  Graph g;
  to_graph(n, row_ptr, col, weight, g);
  std::vector<int64_t> gv(gid, gid + n);
  std::vector<AmgLevel> lv = amg_setup(g, gv);
  Vec fv(f, f + n), uv;
  vcycle(lv, 0, fv, sigma, nsmooth, uv);
  std::copy(uv.begin(), uv.end(), u);
  return 0;
}

int orc_partition(int64_t nelem, int32_t nv, const int64_t *ids, int32_t nparts, const orc_opts *o,
                  int32_t *part, orc_info *info) {
  if (!valid_mesh(nelem, nv, ids) || nparts < 1 || nparts > nelem || !o || !part) return -1;
  Graph g = build_dual_graph(nelem, nv, ids, o->graph);
  std::vector<int64_t> all(nelem);
  for (int64_t i = 0; i < nelem; ++i) all[i] = i;
  orc_info li{};
  int worst = 0;
  WarmMap warm;
  if (o->bfs_start) bfs_start_values(g, all, warm);
  int r = rsb_recurse(g, all, 0, nparts, *o, part, li, worst, warm, true);
  if (info) *info = li;
  if (r < 0) return r;
  return worst;
}

int orc_metrics(int64_t nelem, int32_t nv, const int64_t *ids, int32_t nparts, const int32_t *part,
                double *out) {
  if (!valid_mesh(nelem, nv, ids) || nparts < 1 || !part || !out) return -1;
  Graph g = build_dual_graph(nelem, nv, ids, ORC_GRAPH_WEIGHTED);
  double wcut = 0.0, pairs = 0.0;
  std::vector<std::set<int32_t>> nbr(nparts);
  std::vector<int64_t> sizes(nparts, 0);
  for (int64_t i = 0; i < nelem; ++i) {
    if (part[i] < 0 || part[i] >= nparts) return -1;
    sizes[part[i]] += 1;
    for (auto &nw : g.adj[i])
      if (part[nw.first] != part[i]) {
        nbr[part[i]].insert(part[nw.first]);
        if (nw.first > i) {
          wcut += nw.second;
          pairs += 1.0;
        }
      }
  }
  double mx = 0.0, sum = 0.0;
  for (auto &s : nbr) {
    mx = std::max(mx, (double)s.size());
    sum += (double)s.size();
  }
  out[0] = wcut;
  out[1] = pairs;
  out[2] = mx;
  out[3] = sum / nparts;
  out[4] = (double)*std::min_element(sizes.begin(), sizes.end());
  out[5] = (double)*std::max_element(sizes.begin(), sizes.end());
  return 0;
}

}  // extern "C"
