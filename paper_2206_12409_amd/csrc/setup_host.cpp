// Host-side setup: Gauss tables, RWG tables and ports, pFFT stencils and projection weights,
// extended grid, small dense linear algebra, thread pool helper.
#include <algorithm>
#include <cmath>
#include <map>
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

void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn) {
  if (nthreads <= 1 || n < 64) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&fn, a, b]() { fn(a, b); });
  }
  for (auto& x : th) x.join();
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
void qr_mgs2(std::vector<cxd>& A, int m, int n, std::vector<cxd>& Rm) {
  // Classical Gram-Schmidt applied twice; a column that is numerically dependent on the previous
  // ones is replaced by a fixed pseudo-random vector (then orthogonalised), so Q always has full
  // column rank and the maximum-volume submatrix stays invertible.
  Rm.assign((size_t)n * n, cxd{0, 0});
  double maxnorm = 0;
  for (int j = 0; j < n; ++j) {
    double c = 0;
    for (int r = 0; r < m; ++r) c += A[(size_t)r * n + j].re * A[(size_t)r * n + j].re + A[(size_t)r * n + j].im * A[(size_t)r * n + j].im;
    maxnorm = std::max(maxnorm, sqrt(c));
  }
  uint64_t state = 0x9E3779B97F4A7C15ull;
  for (int j = 0; j < n; ++j) {
    for (int attempt = 0; attempt < 3; ++attempt) {
      double before = 0;
      for (int r = 0; r < m; ++r) before += A[(size_t)r * n + j].re * A[(size_t)r * n + j].re + A[(size_t)r * n + j].im * A[(size_t)r * n + j].im;
      before = sqrt(before);
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < j; ++i) {
          cxd d = {0, 0};
          for (int r = 0; r < m; ++r) d += mul_conj_a(A[(size_t)r * n + i], A[(size_t)r * n + j]);
          for (int r = 0; r < m; ++r) A[(size_t)r * n + j] -= d * A[(size_t)r * n + i];
          if (attempt == 0) Rm[(size_t)i * n + j] += d;
        }
      }
      double after = 0;
      for (int r = 0; r < m; ++r) after += A[(size_t)r * n + j].re * A[(size_t)r * n + j].re + A[(size_t)r * n + j].im * A[(size_t)r * n + j].im;
      after = sqrt(after);
      if (after > 1e-12 * std::max(before, maxnorm) && after > 0) break;
      for (int r = 0; r < m; ++r) {
        state ^= state << 13; state ^= state >> 7; state ^= state << 17;
        A[(size_t)r * n + j] = {(double)(state % 2001) / 1000.0 - 1.0, 0.0};
      }
    }
    double nr = 0;
    for (int r = 0; r < m; ++r) nr += A[(size_t)r * n + j].re * A[(size_t)r * n + j].re + A[(size_t)r * n + j].im * A[(size_t)r * n + j].im;
    nr = sqrt(nr);
    Rm[(size_t)j * n + j] = {nr, 0};
    double inv = nr > 0 ? 1.0 / nr : 0.0;
    for (int r = 0; r < m; ++r) A[(size_t)r * n + j] = inv * A[(size_t)r * n + j];
  }
}

bool lu_solve(std::vector<cxd> A, int n, std::vector<cxd>& B, int nrhs) {
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = -1;
    for (int r = c; r < n; ++r) {
      double v = A[(size_t)r * n + c].re * A[(size_t)r * n + c].re + A[(size_t)r * n + c].im * A[(size_t)r * n + c].im;
      if (v > best) { best = v; p = r; }
    }
    if (best <= 0) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)p * n + j]);
      for (int j = 0; j < nrhs; ++j) std::swap(B[(size_t)c * nrhs + j], B[(size_t)p * nrhs + j]);
    }
    cxd inv = cinv(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      cxd f = A[(size_t)r * n + c] * inv;
      if (f.re == 0 && f.im == 0) continue;
      for (int j = c; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
      for (int j = 0; j < nrhs; ++j) B[(size_t)r * nrhs + j] -= f * B[(size_t)c * nrhs + j];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    cxd inv = cinv(A[(size_t)c * n + c]);
    for (int j = 0; j < nrhs; ++j) {
      cxd s = B[(size_t)c * nrhs + j];
      for (int k = c + 1; k < n; ++k) s -= A[(size_t)c * n + k] * B[(size_t)k * nrhs + j];
      B[(size_t)c * nrhs + j] = s * inv;
    }
  }
  return true;
}

// maxvol: r rows of the m x r matrix Q forming a submatrix of (locally) maximal volume.
std::vector<int> maxvol(const std::vector<cxd>& Q, int m, int r) {
  std::vector<int> rows;
  // greedy start: pivoted Gaussian elimination on a copy
  std::vector<cxd> A = Q;
  std::vector<int> perm(m);
  for (int i = 0; i < m; ++i) perm[i] = i;
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
    cxd inv = cinv(A[(size_t)c * r + c]);
    for (int i = c + 1; i < m; ++i) {
      cxd f = A[(size_t)i * r + c] * inv;
      for (int j = c; j < r; ++j) A[(size_t)i * r + j] -= f * A[(size_t)c * r + j];
    }
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
  for (int it = 0; it < 200; ++it) {
    double best = 0;
    int bi = -1, bj = -1;
    for (int a = 0; a < r; ++a)
      for (int i = 0; i < m; ++i) {
        cxd v = BT[(size_t)a * m + i];
        double av = v.re * v.re + v.im * v.im;
        if (av > best) { best = av; bi = i; bj = a; }
      }
    if (best <= (1.0 + 1e-2) * (1.0 + 1e-2) || bi < 0) break;
    cxd piv = BT[(size_t)bj * m + bi];
    cxd ipiv = cinv(piv);
    std::vector<cxd> col(m), rowv(r);
    for (int i = 0; i < m; ++i) col[i] = BT[(size_t)bj * m + i];                   // B[:, j]
    for (int a = 0; a < r; ++a) rowv[a] = BT[(size_t)a * m + bi];                  // B[i, :]
    rowv[bj] -= cxd{1.0, 0.0};
    for (int a = 0; a < r; ++a) {
      cxd f = rowv[a] * ipiv;
      if (f.re == 0 && f.im == 0) continue;
      for (int i = 0; i < m; ++i) BT[(size_t)a * m + i] -= col[i] * f;
    }
    rows[bj] = bi;
  }
  return rows;
}

}  // namespace vsie
