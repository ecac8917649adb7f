// Host-side setup: Gauss tables, RWG tables and ports, pFFT stencils and projection weights,
// extended grid, small dense linear algebra, thread pool helper.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>

#include "vsie_internal.h"

namespace vsie {

void fill_gauss_table(GaussTab* t) {
  for (int n = 0; n <= GMAX; ++n)
    for (int i = 0; i < GMAX; ++i) t->x[n][i] = t->w[n][i] = 0.0;
  for (int n = 1; n <= GMAX; ++n) {
    for (int i = 0; i < n; ++i) {
      // Newton on P_n from the Chebyshev-like initial guess
      long double x = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
      long double dp = 0;
      for (int it = 0; it < 100; ++it) {
        long double p0 = 1, p1 = x;
        for (int k = 2; k <= n; ++k) {
          long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        if (n == 1) { p1 = x; p0 = 1; }
        dp = n * (x * p1 - p0) / (x * x - 1);
        long double dx = p1 / dp;
        x -= dx;
        if (fabsl(dx) < 1e-19L) break;
      }
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1; }
      dp = n * (x * p1 - p0) / (x * x - 1);
      long double w = 2.0L / ((1 - x * x) * dp * dp);
      // map [-1,1] -> [0,1]
      t->x[n][i] = (double)(0.5L * (1.0L - x));
      t->w[n][i] = (double)(0.5L * w);
    }
  }
}

// Persistent workers for parallel_for: the setup loops call it thousands of times (the TT-cross
// linear algebra once per column), so threads are started once and woken per call.
namespace {
thread_local bool t_in_pool = false;   // set while a thread runs parallel_for work
class Workers {
 public:
  explicit Workers(int n) {
    for (int w = 1; w < n; ++w) th_.emplace_back([this, w]() { loop(w); });
  }
  ~Workers() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  int size() const { return (int)th_.size() + 1; }
  // chunk w of [0, n) for w < parts on worker w (the caller takes chunk 0); returns when all ran
  void run(int64_t n, int parts, const std::function<void(int64_t, int64_t)>& fn) {
    std::unique_lock<std::mutex> lk(call_mu_);   // one call at a time
    {
      std::lock_guard<std::mutex> g(mu_);
      fn_ = &fn;
      n_ = n;
      parts_ = parts;
      chunk_ = (n + parts - 1) / parts;
      pending_ = parts - 1;
      ++gen_;
    }
    cv_.notify_all();
    fn(0, std::min(n, chunk_));
    std::unique_lock<std::mutex> g(mu_);
    done_.wait(g, [this]() { return pending_ == 0; });
  }

 private:
  void loop(int w) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int64_t, int64_t)>* fn;
      int64_t a, b;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&]() { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        if (w >= parts_) continue;
        fn = fn_;
        a = w * chunk_;
        b = std::min(n_, a + chunk_);
      }
      t_in_pool = true;
      if (a < b) (*fn)(a, b);
      t_in_pool = false;
      {
        std::lock_guard<std::mutex> g(mu_);
        if (--pending_ == 0) done_.notify_one();
      }
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_, call_mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int64_t, int64_t)>* fn_ = nullptr;
  int64_t n_ = 0, chunk_ = 0;
  int parts_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};
}  // namespace

void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn) {
  static Workers pool(host_threads());
  const int parts = (int)std::min<int64_t>(std::min(nthreads, pool.size()), n);
  if (parts <= 1 || t_in_pool) {   // nested calls run inline
    fn(0, n);
    return;
  }
  t_in_pool = true;
  pool.run(n, parts, fn);
  t_in_pool = false;
}

int host_threads() {
  unsigned hc = std::thread::hardware_concurrency();
  if (hc == 0) hc = 4;
  return (int)std::min<unsigned>(hc, 16);
}

// ---------------------------------------------------------------------------------------------
// RWG tables for all meshes of one domain, concatenated in input order.
void build_rwg(const vsie_problem* p, int domain, Rwg& R,
               std::vector<std::pair<int, std::vector<PortEdge>>>& ports) {
  std::vector<int> voff(p->n_meshes, -1);
  int nv = 0;
  for (int mi = 0; mi < p->n_meshes; ++mi) {
    const vsie_mesh& m = p->meshes[mi];
    if (m.domain != domain) continue;
    if (m.n_verts <= 0 || m.n_tris <= 0 || !m.verts || !m.tris) throw Error(VSIE_E_ARG, "empty mesh");
    voff[mi] = nv;
    for (int i = 0; i < 3 * m.n_verts; ++i) {
      if (!std::isfinite(m.verts[i])) throw Error(VSIE_E_ARG, "non-finite vertex coordinate");
      R.verts.push_back(m.verts[i]);
    }
    for (int i = 0; i < 3 * m.n_tris; ++i) {
      int v = m.tris[i];
      if (v < 0 || v >= m.n_verts) throw Error(VSIE_E_MESH, "triangle vertex id out of range");
      R.tris.push_back(v + nv);
    }
    nv += m.n_verts;
  }
  const int nt = (int)R.tris.size() / 3;
  R.area.resize(nt);
  for (int t = 0; t < nt; ++t) {
    V3 a = R.vert(R.tris[3 * t]), b = R.vert(R.tris[3 * t + 1]), c = R.vert(R.tris[3 * t + 2]);
    R.area[t] = 0.5 * norm(cross(b - a, c - a));
    if (!(R.area[t] > 0)) throw Error(VSIE_E_MESH, "degenerate triangle");
  }
  // directed edge -> (triangle, local index of the opposite vertex)
  std::map<std::pair<int, int>, std::pair<int, int>> dir;
  for (int t = 0; t < nt; ++t) {
    int v[3] = {R.tris[3 * t], R.tris[3 * t + 1], R.tris[3 * t + 2]};
    for (int e = 0; e < 3; ++e) {
      int a = v[e], b = v[(e + 1) % 3];
      int fl = (e + 2) % 3;
      auto key = std::make_pair(a, b);
      if (dir.count(key)) throw Error(VSIE_E_MESH, "inconsistent orientation or non-manifold edge");
      dir[key] = std::make_pair(t, fl);
    }
  }
  for (auto& kv : dir) {
    int a = kv.first.first, b = kv.first.second;
    if (a > b) continue;
    auto it = dir.find(std::make_pair(b, a));
    if (it == dir.end()) continue;   // boundary edge
    int tp = kv.second.first, flp = kv.second.second;
    int tm = it->second.first, flm = it->second.second;
    R.ea.push_back(a);
    R.eb.push_back(b);
    R.tp.push_back(tp);
    R.tm.push_back(tm);
    R.flp.push_back(flp);
    R.flm.push_back(flm);
    R.fp.push_back(R.tris[3 * tp + flp]);
    R.fm.push_back(R.tris[3 * tm + flm]);
    R.len.push_back(norm(R.vert(b) - R.vert(a)));
  }
  R.m = (int)R.ea.size();   // std::map iterates in (a, b) order: edges sorted by (min, max)
  // ports, mesh by mesh
  std::map<std::pair<int, int>, int> lookup;
  for (int i = 0; i < R.m; ++i) lookup[std::make_pair(R.ea[i], R.eb[i])] = i;
  for (int mi = 0; mi < p->n_meshes; ++mi) {
    const vsie_mesh& m = p->meshes[mi];
    if (m.domain != domain || m.n_port_edges <= 0) continue;
    int np = 0;
    for (int e = 0; e < m.n_port_edges; ++e) np = std::max(np, m.port_id[e] + 1);
    std::vector<std::vector<PortEdge>> mp(np);
    for (int e = 0; e < m.n_port_edges; ++e) {
      int a = m.port_edges[2 * e] + voff[mi], b = m.port_edges[2 * e + 1] + voff[mi];
      auto key = std::make_pair(std::min(a, b), std::max(a, b));
      auto it = lookup.find(key);
      if (it == lookup.end()) throw Error(VSIE_E_MESH, "port edge is not an interior edge");
      if (m.port_id[e] < 0) throw Error(VSIE_E_ARG, "negative port id");
      mp[m.port_id[e]].push_back(PortEdge{domain, it->second, a < b ? 1.0 : -1.0});
    }
    for (auto& x : mp) ports.push_back(std::make_pair(mi, x));
  }
}

// ---------------------------------------------------------------------------------------------
// pFFT stencils. Base voxel: the 5^3 block centred on the voxel containing the midpoint of the
// RWG's common edge; weights reproduce all moments x^a y^b z^c, 0 <= a,b,c <= 4, of the RWG
// current with PWC voxel currents (per axis a 5x5 histopolation system).
static void dual_polys(double C[5][5]) {
  // A[k][i] = int over voxel i of xi^k, xi in [-2.5, 2.5]; C = A^{-1} (rows: polynomial j)
  long double A[5][10];
  for (int k = 0; k < 5; ++k) {
    for (int i = 0; i < 5; ++i) {
      long double a = -2.5L + i, b = a + 1.0L;
      A[k][i] = (powl(b, k + 1) - powl(a, k + 1)) / (k + 1);
    }
    for (int i = 0; i < 5; ++i) A[k][5 + i] = (k == i) ? 1.0L : 0.0L;
  }
  for (int c = 0; c < 5; ++c) {
    int piv = c;
    for (int r = c + 1; r < 5; ++r)
      if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
    for (int j = 0; j < 10; ++j) std::swap(A[c][j], A[piv][j]);
    long double d = A[c][c];
    for (int j = 0; j < 10; ++j) A[c][j] /= d;
    for (int r = 0; r < 5; ++r) {
      if (r == c) continue;
      long double f = A[r][c];
      for (int j = 0; j < 10; ++j) A[r][j] -= f * A[c][j];
    }
  }
  for (int j = 0; j < 5; ++j)
    for (int k = 0; k < 5; ++k) C[j][k] = (double)A[j][5 + k];
}

void stencil_setup(Handle& H) {
  const Rwg& R = H.near;
  const int m = R.m;
  H.base.assign(3 * m, 0);
  int lo[3] = {0, 0, 0}, hi[3] = {H.n[0], H.n[1], H.n[2]};
  for (int i = 0; i < m; ++i) {
    V3 a = R.vert(R.ea[i]), b = R.vert(R.eb[i]);
    double c[3] = {0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z)};
    for (int ax = 0; ax < 3; ++ax) {
      double q = (c[ax] - H.origin[ax]) / H.h;
      if (!std::isfinite(q) || fabs(q) > 1e8) throw Error(VSIE_E_GRID, "near conductor far outside the grid");
      int k = (int)floor(q);
      H.base[3 * i + ax] = k - 2;
    }
    // fit check: both triangles inside [origin + base h, origin + base h + 5 h]
    for (int side = 0; side < 2; ++side) {
      int t = side == 0 ? R.tp[i] : R.tm[i];
      for (int v = 0; v < 3; ++v) {
        V3 p = R.vert(R.tris[3 * t + v]);
        double pc[3] = {p.x, p.y, p.z};
        for (int ax = 0; ax < 3; ++ax) {
          double l = H.origin[ax] + H.base[3 * i + ax] * H.h;
          double u = l + 5 * H.h;
          if (pc[ax] < l || pc[ax] > u)
            throw Error(VSIE_E_STENCIL, "an RWG pair does not fit its 5x5x5 expansion block");
        }
      }
    }
    for (int ax = 0; ax < 3; ++ax) {
      lo[ax] = std::min(lo[ax], H.base[3 * i + ax]);
      hi[ax] = std::max(hi[ax], H.base[3 * i + ax] + 5);
    }
  }
  for (int ax = 0; ax < 3; ++ax) {
    H.ne[ax] = hi[ax] - lo[ax];
    H.ob[ax] = -lo[ax];
    int P = 8;
    while (P < 2 * H.ne[ax] - 1) P *= 2;
    if (P > 1024) throw Error(VSIE_E_GRID, "extended grid needs an FFT longer than 1024");
    H.P[ax] = P;
  }
  H.Ne = (int64_t)H.ne[0] * H.ne[1] * H.ne[2];

  // projection weights by an exact collapsed Gauss rule (9 x 9 points: exact to degree 16;
  // the integrand has degree 13)
  GaussTab gt;
  fill_gauss_table(&gt);
  const int nq = 9;
  std::vector<double> ql1, ql2, ql3, qw;
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b) {
      double u = gt.x[nq][a], s = gt.x[nq][b];
      ql2.push_back(u);
      ql3.push_back(s * (1.0 - u));
      ql1.push_back(1.0 - u - s * (1.0 - u));
      qw.push_back(2.0 * gt.w[nq][a] * gt.w[nq][b] * (1.0 - u));
    }
  double C[5][5];
  dual_polys(C);
  H.Wh.assign((size_t)m * 375, 0.0);
  const double h3 = H.h * H.h * H.h;
  parallel_for(m, host_threads(), [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      double cen[3];
      for (int ax = 0; ax < 3; ++ax) cen[ax] = H.origin[ax] + (H.base[3 * i + ax] + 2.5) * H.h;
      double* W = &H.Wh[(size_t)i * 375];
      for (int side = 0; side < 2; ++side) {
        int t = side == 0 ? R.tp[i] : R.tm[i];
        int fv = side == 0 ? R.fp[i] : R.fm[i];
        double s = side == 0 ? 1.0 : -1.0;
        V3 v0 = R.vert(R.tris[3 * t]), v1 = R.vert(R.tris[3 * t + 1]), v2 = R.vert(R.tris[3 * t + 2]);
        V3 pf = R.vert(fv);
        double A = R.area[t];
        double coef = s * R.len[i] / (2.0 * A);
        for (size_t q = 0; q < qw.size(); ++q) {
          V3 r = ql1[q] * v0 + ql2[q] * v1 + ql3[q] * v2;
          V3 f = coef * (r - pf);
          double wA = qw[q] * A;
          double xi[3] = {(r.x - cen[0]) / H.h, (r.y - cen[1]) / H.h, (r.z - cen[2]) / H.h};
          double ph[3][5];
          for (int ax = 0; ax < 3; ++ax)
            for (int j = 0; j < 5; ++j) {
              double v = 0, pw = 1;
              for (int k = 0; k < 5; ++k) {
                v += C[j][k] * pw;
                pw *= xi[ax];
              }
              ph[ax][j] = v;
            }
          const double fc[3] = {f.x, f.y, f.z};
          for (int j3 = 0; j3 < 5; ++j3)
            for (int j2 = 0; j2 < 5; ++j2)
              for (int j1 = 0; j1 < 5; ++j1) {
                double b = wA * ph[0][j1] * ph[1][j2] * ph[2][j3];
                int o = j3 * 25 + j2 * 5 + j1;
                W[0 * 125 + o] += fc[0] * b;
                W[1 * 125 + o] += fc[1] * b;
                W[2 * 125 + o] += fc[2] * b;
              }
        }
      }
      for (int o = 0; o < 375; ++o) W[o] /= h3;
    }
  });
}

// ---------------------------------------------------------------------------------------------
// Small dense complex linear algebra for TT-cross and ACA.
// Row chunks for the host threads of a dense kernel over m rows (at least 2048 rows each).
static int row_threads(int64_t m) { return (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), m / 2048)); }

void qr_mgs2(std::vector<cxd>& A, int m, int n, std::vector<cxd>& Rm) {
  // Classical Gram-Schmidt applied twice; a column that is numerically dependent on the previous
  // ones is replaced by a fixed pseudo-random vector (then orthogonalised), so Q always has full
  // column rank and the maximum-volume submatrix stays invertible. The columns are worked on in a
  // column-major copy (contiguous dot products and updates), the rows split over host threads.
  Rm.assign((size_t)n * n, cxd{0, 0});
  std::vector<cxd> Q((size_t)m * n);
  for (int r = 0; r < m; ++r)
    for (int j = 0; j < n; ++j) Q[(size_t)j * m + r] = A[(size_t)r * n + j];
  const int nt = row_threads(m);
  const int64_t chunk = (m + nt - 1) / nt;
  auto norm2 = [&](const cxd* q) {
    std::vector<double> part(nt, 0.0);
    parallel_for(nt, nt, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t) {
        double acc = 0;
        for (int64_t r = t * chunk; r < std::min<int64_t>(m, (t + 1) * chunk); ++r) acc += q[r].re * q[r].re + q[r].im * q[r].im;
        part[t] = acc;
      }
    });
    double s2 = 0;
    for (double v : part) s2 += v;
    return s2;
  };
  double maxnorm = 0;
  for (int j = 0; j < n; ++j) maxnorm = std::max(maxnorm, sqrt(norm2(&Q[(size_t)j * m])));
  uint64_t state = 0x9E3779B97F4A7C15ull;
  std::vector<cxd> part((size_t)nt * std::max(n, 1)), d(std::max(n, 1));
  for (int j = 0; j < n; ++j) {
    cxd* qj = &Q[(size_t)j * m];
    for (int attempt = 0; attempt < 3; ++attempt) {
      const double before = sqrt(norm2(qj));
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        // d = Q[:, :j]^H q_j (partial sums per row chunk), then q_j -= Q[:, :j] d
        parallel_for(nt, nt, [&](int64_t t0, int64_t t1) {
          for (int64_t t = t0; t < t1; ++t) {
            const int64_t r0 = t * chunk, r1 = std::min<int64_t>(m, r0 + chunk);
            for (int i = 0; i < j; ++i) {
              const cxd* qi = &Q[(size_t)i * m];
              cxd acc = {0, 0};
              for (int64_t r = r0; r < r1; ++r) acc += mul_conj_a(qi[r], qj[r]);
              part[(size_t)t * n + i] = acc;
            }
          }
        });
        for (int i = 0; i < j; ++i) {
          cxd acc = {0, 0};
          for (int t = 0; t < nt; ++t) acc += part[(size_t)t * n + i];
          d[i] = acc;
          if (attempt == 0) Rm[(size_t)i * n + j] += acc;
        }
        parallel_for(nt, nt, [&](int64_t t0, int64_t t1) {
          for (int64_t t = t0; t < t1; ++t) {
            const int64_t r0 = t * chunk, r1 = std::min<int64_t>(m, r0 + chunk);
            for (int i = 0; i < j; ++i) {
              const cxd* qi = &Q[(size_t)i * m];
              const cxd di = d[i];
              for (int64_t r = r0; r < r1; ++r) qj[r] -= di * qi[r];
            }
          }
        });
      }
      const double after = sqrt(norm2(qj));
      if (after > 1e-12 * std::max(before, maxnorm) && after > 0) break;
      for (int r = 0; r < m; ++r) {
        state ^= state << 13; state ^= state >> 7; state ^= state << 17;
        qj[r] = {(double)(state % 2001) / 1000.0 - 1.0, 0.0};
      }
    }
    const double nr = sqrt(norm2(qj));
    Rm[(size_t)j * n + j] = {nr, 0};
    const double inv = nr > 0 ? 1.0 / nr : 0.0;
    for (int r = 0; r < m; ++r) qj[r] = inv * qj[r];
  }
  for (int r = 0; r < m; ++r)
    for (int j = 0; j < n; ++j) A[(size_t)r * n + j] = Q[(size_t)j * m + r];
}

bool lu_solve(std::vector<cxd> A, int n, std::vector<cxd>& B, int nrhs) {
  // partial pivoting on A (row-major n x n); every row operation on B (n x nrhs, row-major) is a
  // contiguous sweep, the right-hand sides split over host threads
  std::vector<int> piv(n);
  std::vector<cxd> F((size_t)n * n, cxd{0, 0});   // multipliers, applied to B afterwards
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = -1;
    for (int r = c; r < n; ++r) {
      double v = A[(size_t)r * n + c].re * A[(size_t)r * n + c].re + A[(size_t)r * n + c].im * A[(size_t)r * n + c].im;
      if (v > best) { best = v; p = r; }
    }
    if (best <= 0) return false;
    piv[c] = p;
    if (p != c)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)p * n + j]);
    const cxd inv = cinv(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      const cxd f = A[(size_t)r * n + c] * inv;
      F[(size_t)r * n + c] = f;
      if (f.re == 0 && f.im == 0) continue;
      for (int j = c; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
    }
  }
  const int nt = row_threads(nrhs);
  const int64_t chunk = (nrhs + nt - 1) / nt;
  parallel_for(nt, nt, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t j0 = t * chunk, j1 = std::min<int64_t>(nrhs, j0 + chunk);
      if (j0 >= j1) continue;
      for (int c = 0; c < n; ++c) {
        if (piv[c] != c)
          for (int64_t j = j0; j < j1; ++j) std::swap(B[(size_t)c * nrhs + j], B[(size_t)piv[c] * nrhs + j]);
        for (int r = c + 1; r < n; ++r) {
          const cxd f = F[(size_t)r * n + c];
          if (f.re == 0 && f.im == 0) continue;
          for (int64_t j = j0; j < j1; ++j) B[(size_t)r * nrhs + j] -= f * B[(size_t)c * nrhs + j];
        }
      }
      for (int c = n - 1; c >= 0; --c) {
        for (int k = c + 1; k < n; ++k) {
          const cxd a = A[(size_t)c * n + k];
          for (int64_t j = j0; j < j1; ++j) B[(size_t)c * nrhs + j] -= a * B[(size_t)k * nrhs + j];
        }
        const cxd inv = cinv(A[(size_t)c * n + c]);
        for (int64_t j = j0; j < j1; ++j) B[(size_t)c * nrhs + j] = B[(size_t)c * nrhs + j] * inv;
      }
    }
  });
  return true;
}

std::vector<int> maxvol(const std::vector<cxd>& Q, int m, int r) {
  std::vector<int> rows;
  // greedy start: pivoted Gaussian elimination on a copy (row updates split over host threads)
  std::vector<cxd> A = Q;
  std::vector<int> perm(m);
  for (int i = 0; i < m; ++i) perm[i] = i;
  const int nt = row_threads(m);
  for (int c = 0; c < r; ++c) {
    int p = c;
    double best = -1;
    for (int i = c; i < m; ++i) {
      cxd v = A[(size_t)i * r + c];
      double a = v.re * v.re + v.im * v.im;
      if (a > best) { best = a; p = i; }
    }
    std::swap(perm[c], perm[p]);
    for (int j = 0; j < r; ++j) std::swap(A[(size_t)c * r + j], A[(size_t)p * r + j]);
    if (best <= 0) continue;
    const cxd inv = cinv(A[(size_t)c * r + c]);
    parallel_for(m - c - 1, nt, [&](int64_t a0, int64_t a1) {
      for (int64_t i = c + 1 + a0; i < c + 1 + a1; ++i) {
        const cxd f = A[(size_t)i * r + c] * inv;
        for (int j = c; j < r; ++j) A[(size_t)i * r + j] -= f * A[(size_t)c * r + j];
      }
    });
  }
  rows.assign(perm.begin(), perm.begin() + r);
  // refinement: B = Q Q_rows^{-1} (m x r); while some |B[i][j]| > 1 + 1e-2 swap row i into
  // position j and update B with the rank-one correction B -= B[:, j] (B[i, :] - e_j) / B[i][j].
  std::vector<cxd> S((size_t)r * r), BT((size_t)r * m);
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) S[(size_t)a * r + b] = Q[(size_t)rows[b] * r + a];   // S = Q_rows^T
  for (int a = 0; a < r; ++a)
    for (int i = 0; i < m; ++i) BT[(size_t)a * m + i] = Q[(size_t)i * r + a];
  if (!lu_solve(S, r, BT, m)) return rows;                                          // BT = B^T
  // the search and the rank-one update run over rows of B^T split among host threads; ties go
  // to the lowest (a, i) as in a sequential scan
  const int ntr = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)host_threads(), (int64_t)r,
                                                                (int64_t)m * r / 65536}));
  std::vector<double> tbest(ntr);
  std::vector<int> tbi(ntr), tbj(ntr);
  std::vector<cxd> col(m), rowv(r);
  for (int it = 0; it < 200; ++it) {
    parallel_for(ntr, ntr, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t) {
        double best = 0;
        int bi = -1, bj = -1;
        for (int a = (int)(t * r / ntr); a < (int)((t + 1) * r / ntr); ++a)
          for (int i = 0; i < m; ++i) {
            const cxd v = BT[(size_t)a * m + i];
            const double av = v.re * v.re + v.im * v.im;
            if (av > best) { best = av; bi = i; bj = a; }
          }
        tbest[t] = best;
        tbi[t] = bi;
        tbj[t] = bj;
      }
    });
    double best = 0;
    int bi = -1, bj = -1;
    for (int t = 0; t < ntr; ++t)
      if (tbest[t] > best) { best = tbest[t]; bi = tbi[t]; bj = tbj[t]; }
    if (best <= (1.0 + 1e-2) * (1.0 + 1e-2) || bi < 0) break;
    const cxd ipiv = cinv(BT[(size_t)bj * m + bi]);
    for (int i = 0; i < m; ++i) col[i] = BT[(size_t)bj * m + i];                   // B[:, j]
    for (int a = 0; a < r; ++a) rowv[a] = BT[(size_t)a * m + bi];                  // B[i, :]
    rowv[bj] -= cxd{1.0, 0.0};
    parallel_for(ntr, ntr, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t)
        for (int a = (int)(t * r / ntr); a < (int)((t + 1) * r / ntr); ++a) {
          const cxd f = rowv[a] * ipiv;
          if (f.re == 0 && f.im == 0) continue;
          for (int i = 0; i < m; ++i) BT[(size_t)a * m + i] -= col[i] * f;
        }
    });
    rows[bj] = bi;
  }
  return rows;
}


}  // namespace vsie
