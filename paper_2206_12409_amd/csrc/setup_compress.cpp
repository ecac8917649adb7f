// TT-cross of a 4D tensor given by an entry function (paper Sec. II-D, Sec. III eq. (14)).
//
// Interpolative TT construction from sampled fibres: nested left index sets I_k (multi-indices
// over i_1..i_k) and right index sets J_k (over i_{k+1}..i_4) are refined by alternating sweeps;
// at every step the fibre matrix C_k = A(I_{k-1}, i_k, J_k) is orthogonalised (QR) and its
// maximum-volume rows give the next index set. Cores follow from the cross interpolation
// formula G_k = Q_k Q_k[rows]^{-1}, G_4 = A(I_3, i_4). Ranks grow (with random enrichment of the
// index sets) until the relative error measured on random held-out entries is below the
// tolerance or the rank cap is reached; a rank stops growing once its fibre matrix is
// numerically rank deficient at the tolerance. The paper uses the two-site DMRG variant of TT-cross;
// this one-site variant with explicit rank growth reaches the same accuracy target.
#include <algorithm>
#include <cmath>
#include <random>

#include "vsie_internal.h"

namespace vsie {

namespace {

using Multi = std::vector<int>;   // flattened multi-indices, fixed arity per set

struct Sets {
  std::vector<Multi> I;   // I[k]: left multi-indices of arity k+1 (k = 0..2), as tuples
  std::vector<Multi> J;   // J[k]: right multi-indices over i_{k+2}..i_4 (k = 0..2)
};

// evaluate the (r_left * n_k) x r_right fibre matrix; rows (a, i) with a fastest? -> row = a * n + i
void fibre(EntryFn& f, const std::vector<std::vector<int>>& left, int nk, int k,
           const std::vector<std::vector<int>>& right, std::vector<cxd>& C) {
  const size_t rl = left.size(), rr = right.size();
  std::vector<int> idx;
  idx.reserve(rl * nk * rr * 4);
  for (size_t a = 0; a < rl; ++a)
    for (int i = 0; i < nk; ++i)
      for (size_t b = 0; b < rr; ++b) {
        int t[4];
        int p = 0;
        for (int v : left[a]) t[p++] = v;
        t[p++] = i;
        for (int v : right[b]) t[p++] = v;
        (void)k;
        for (int q = 0; q < 4; ++q) idx.push_back(t[q]);
      }
  f.eval(idx, C);   // C[(a * nk + i) * rr + b]
}

// sigma_min / sigma_max of an m x n complex matrix (row-major, m >= n) from the eigenvalues of
// its Gram matrix C^H C, computed by cyclic Jacobi on the equivalent real symmetric 2n x 2n
// matrix [[Re, -Im], [Im, Re]] (each eigenvalue appears twice). Resolves ratios down to ~1e-7.
double sv_ratio(const std::vector<cxd>& C, int m, int n) {
  if (n <= 1) return 1.0;
  std::vector<cxd> G((size_t)n * n, cxd{0, 0});
  for (int r = 0; r < m; ++r) {
    const cxd* row = &C[(size_t)r * n];
    for (int a = 0; a < n; ++a)
      for (int b = a; b < n; ++b) G[(size_t)a * n + b] += mul_conj_a(row[a], row[b]);
  }
  const int N2 = 2 * n;
  std::vector<double> S((size_t)N2 * N2);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const cxd g = a <= b ? G[(size_t)a * n + b] : cxd{G[(size_t)b * n + a].re, -G[(size_t)b * n + a].im};
      S[(size_t)a * N2 + b] = g.re;
      S[(size_t)(a + n) * N2 + (b + n)] = g.re;
      S[(size_t)(a + n) * N2 + b] = g.im;
      S[(size_t)a * N2 + (b + n)] = -g.im;
    }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0, diag = 0;
    for (int i = 0; i < N2; ++i) {
      diag += S[(size_t)i * N2 + i] * S[(size_t)i * N2 + i];
      for (int j = i + 1; j < N2; ++j) off += S[(size_t)i * N2 + j] * S[(size_t)i * N2 + j];
    }
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < N2; ++p)
      for (int q = p + 1; q < N2; ++q) {
        const double apq = S[(size_t)p * N2 + q];
        if (apq == 0) continue;
        const double app = S[(size_t)p * N2 + p], aqq = S[(size_t)q * N2 + q];
        const double theta = (aqq - app) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), sn = t * c;
        for (int k = 0; k < N2; ++k) {   // S <- J^T S J on rows/columns p, q
          const double skp = S[(size_t)k * N2 + p], skq = S[(size_t)k * N2 + q];
          S[(size_t)k * N2 + p] = c * skp - sn * skq;
          S[(size_t)k * N2 + q] = sn * skp + c * skq;
        }
        for (int k = 0; k < N2; ++k) {
          const double spk = S[(size_t)p * N2 + k], sqk = S[(size_t)q * N2 + k];
          S[(size_t)p * N2 + k] = c * spk - sn * sqk;
          S[(size_t)q * N2 + k] = sn * spk + c * sqk;
        }
      }
  }
  double lmax = 0, lmin = 1e300;
  for (int i = 0; i < N2; ++i) {
    lmax = std::max(lmax, S[(size_t)i * N2 + i]);
    lmin = std::min(lmin, S[(size_t)i * N2 + i]);
  }
  if (lmax <= 0) return 0.0;
  return std::sqrt(std::max(lmin, 0.0) / lmax);
}

// Eigen-decomposition of a Hermitian n x n matrix (row-major) by cyclic complex Jacobi rotations:
// H = V diag(w) V^H, V unitary (row-major, column j the j-th eigenvector).
void herm_eig(std::vector<cxd> A, int n, std::vector<double>& w, std::vector<cxd>& V) {
  V.assign((size_t)n * n, cxd{0, 0});
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = {1, 0};
  auto at = [&](int r, int c) -> cxd& { return A[(size_t)r * n + c]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, dg = 0;
    for (int i = 0; i < n; ++i) {
      dg += at(i, i).re * at(i, i).re;
      for (int j = i + 1; j < n; ++j) off += at(i, j).re * at(i, j).re + at(i, j).im * at(i, j).im;
    }
    if (off <= 1e-30 * dg) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cxd apq = at(p, q);
        const double mag = std::sqrt(apq.re * apq.re + apq.im * apq.im);
        if (mag == 0) continue;
        // e = exp(-i arg(a_pq)) turns the pair real; then a real rotation (c, s) zeroes it
        const cxd e = {apq.re / mag, -apq.im / mag};
        const cxd ec = {e.re, -e.im};
        const double th = (at(q, q).re - at(p, p).re) / (2 * mag);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double c = 1 / std::sqrt(t * t + 1), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const cxd xp = at(k, p), xq = at(k, q) * e;
          at(k, p) = c * xp - sn * xq;
          at(k, q) = sn * xp + c * xq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const cxd xp = at(p, k), xq = at(q, k) * ec;
          at(p, k) = c * xp - sn * xq;
          at(q, k) = sn * xp + c * xq;
        }
        for (int k = 0; k < n; ++k) {
          const cxd vp = V[(size_t)k * n + p], vq = V[(size_t)k * n + q] * e;
          V[(size_t)k * n + p] = c * vp - sn * vq;
          V[(size_t)k * n + q] = sn * vp + c * vq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = at(i, i).re;
}

// C = A B, A (m x k), B (k x n), row-major
std::vector<cxd> matmul(const std::vector<cxd>& A, const std::vector<cxd>& B, int m, int k, int n) {
  std::vector<cxd> C((size_t)m * n, cxd{0, 0});
  parallel_for(m, host_threads(), [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i)
      for (int l = 0; l < k; ++l) {
        const cxd a = A[(size_t)i * k + l];
        const cxd* b = &B[(size_t)l * n];
        cxd* c = &C[(size_t)i * n];
        for (int j = 0; j < n; ++j) c[j] += a * b[j];
      }
  });
  return C;
}

// M (m x n) = L Q with orthonormal rows of Q (r x n) and L (m x r), from the eigen-decomposition
// of the Gram matrix M M^H = W diag(w) W^H: L = W sqrt(w), Q = diag(1/sqrt(w)) W^H M; directions
// with w at rounding level are dropped (r <= m).
void right_orth(const std::vector<cxd>& M, int m, int n, std::vector<cxd>& L, std::vector<cxd>& Q, int& r) {
  std::vector<cxd> H((size_t)m * m, cxd{0, 0});
  parallel_for(m, host_threads(), [&](int64_t a0, int64_t a1) {
    for (int64_t a = a0; a < a1; ++a)
      for (int b = 0; b < m; ++b) {
        cxd acc = {0, 0};
        for (int j = 0; j < n; ++j) acc += mul_conj_b(M[(size_t)a * n + j], M[(size_t)b * n + j]);
        H[(size_t)a * m + b] = acc;
      }
  });
  std::vector<double> w;
  std::vector<cxd> W;
  herm_eig(H, m, w, W);
  double wmax = 0;
  for (double v : w) wmax = std::max(wmax, v);
  std::vector<int> keep;
  for (int i = 0; i < m; ++i)
    if (w[i] > 1e-28 * wmax && w[i] > 0) keep.push_back(i);
  r = (int)keep.size();
  L.assign((size_t)m * r, cxd{0, 0});
  std::vector<cxd> WH((size_t)r * m);
  for (int j = 0; j < r; ++j) {
    const double sw = std::sqrt(w[keep[j]]);
    for (int i = 0; i < m; ++i) {
      L[(size_t)i * r + j] = sw * W[(size_t)i * m + keep[j]];
      WH[(size_t)j * m + i] = (1.0 / sw) * conj(W[(size_t)i * m + keep[j]]);
    }
  }
  Q = matmul(WH, M, r, m, n);
}

// M (m x n) ~ U S V^H truncated to the smallest rank r whose discarded squared singular values sum
// to at most d2, from the Gram matrix M^H M = V diag(s^2) V^H: U = M V_r / s (orthonormal
// columns, m x r) and SVh = diag(s) V_r^H (r x n).
void left_trunc(const std::vector<cxd>& M, int m, int n, double d2, std::vector<cxd>& U, std::vector<cxd>& SVh,
                int& r) {
  std::vector<cxd> H((size_t)n * n, cxd{0, 0});
  parallel_for(n, host_threads(), [&](int64_t a0, int64_t a1) {
    for (int64_t a = a0; a < a1; ++a)
      for (int b = 0; b < n; ++b) {
        cxd acc = {0, 0};
        for (int i = 0; i < m; ++i) acc += mul_conj_a(M[(size_t)i * n + a], M[(size_t)i * n + b]);
        H[(size_t)a * n + b] = acc;
      }
  });
  std::vector<double> w;
  std::vector<cxd> V;
  herm_eig(H, n, w, V);
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a] > w[b] || (w[a] == w[b] && a < b); });
  r = n;
  double tail = 0;
  for (int i = n - 1; i >= 1; --i) {
    tail += std::max(w[ord[i]], 0.0);
    if (tail > d2) break;
    r = i;
  }
  while (r > 1 && !(w[ord[r - 1]] > 0)) --r;
  std::vector<cxd> Vr((size_t)n * r);
  SVh.assign((size_t)r * n, cxd{0, 0});
  for (int j = 0; j < r; ++j) {
    const double s = std::sqrt(std::max(w[ord[j]], 0.0));
    for (int i = 0; i < n; ++i) {
      Vr[(size_t)i * r + j] = (s > 0 ? 1.0 / s : 0.0) * V[(size_t)i * n + ord[j]];
      SVh[(size_t)j * n + i] = s * conj(V[(size_t)i * n + ord[j]]);
    }
  }
  U = matmul(M, Vr, m, n, r);
}

}  // namespace

// TT rounding: right-to-left orthogonalisation, then left-to-right truncation of each unfolding
// by its singular values with a budget delta^2 ||A||^2 / 3 each, so the rounded train differs
// from the input by at most delta ||A|| in the Frobenius norm.
void tt_round(const int n[4], std::vector<cxd> cores[4], int ranks[3], double delta) {
  int r[3] = {ranks[0], ranks[1], ranks[2]};
  std::vector<cxd> L, Q;
  int rn;
  // G4 = L Q; G3 <- G3 L
  right_orth(cores[3], r[2], n[3], L, Q, rn);
  cores[3] = Q;
  cores[2] = matmul(cores[2], L, r[1] * n[2], r[2], rn);
  r[2] = rn;
  // G3 as r2 x (n3 r3) = L Q; G2 <- G2 L
  right_orth(cores[2], r[1], n[2] * r[2], L, Q, rn);
  cores[2] = Q;
  cores[1] = matmul(cores[1], L, r[0] * n[1], r[1], rn);
  r[1] = rn;
  // G2 as r1 x (n2 r2) = L Q; G1 <- G1 L
  right_orth(cores[1], r[0], n[1] * r[1], L, Q, rn);
  cores[1] = Q;
  cores[0] = matmul(cores[0], L, n[0], r[0], rn);
  r[0] = rn;
  double nrm2 = 0;
  for (const cxd& v : cores[0]) nrm2 += v.re * v.re + v.im * v.im;
  const double d2 = delta * delta * nrm2 / 3.0;
  std::vector<cxd> U, SVh;
  // G1 (n1 x r1) ~ U SVh; G2 <- SVh G2
  left_trunc(cores[0], n[0], r[0], d2, U, SVh, rn);
  cores[0] = U;
  cores[1] = matmul(SVh, cores[1], rn, r[0], n[1] * r[1]);
  r[0] = rn;
  left_trunc(cores[1], r[0] * n[1], r[1], d2, U, SVh, rn);
  cores[1] = U;
  cores[2] = matmul(SVh, cores[2], rn, r[1], n[2] * r[2]);
  r[1] = rn;
  left_trunc(cores[2], r[1] * n[2], r[2], d2, U, SVh, rn);
  cores[2] = U;
  cores[3] = matmul(SVh, cores[3], rn, r[2], n[3]);
  r[2] = rn;
  for (int k = 0; k < 3; ++k) ranks[k] = r[k];
}

void tt_cross(EntryFn& f, const int n[4], double tol, int rmax, uint64_t seed, std::vector<cxd> cores[4],
              int ranks[3], double* err_est) {
  std::mt19937_64 rng(seed);
  // held-out test entries
  const int ntest = 2000;
  std::vector<int> tidx(4 * ntest);
  for (int s = 0; s < ntest; ++s)
    for (int q = 0; q < 4; ++q) tidx[4 * s + q] = (int)(rng() % (uint64_t)n[q]);
  std::vector<cxd> tval;
  f.eval(tidx, tval);
  double tnorm = 0;
  for (auto& v : tval) tnorm += v.re * v.re + v.im * v.im;

  // relative error of a train on the held-out entries
  auto held_out = [&](const std::vector<cxd>* G, const int* rk) {
    double e2 = 0;
    for (int s = 0; s < ntest; ++s) {
      const int* t = &tidx[4 * s];
      std::vector<cxd> v1(rk[0]), v2(rk[1], cxd{0, 0}), v3(rk[2], cxd{0, 0});
      for (int a = 0; a < rk[0]; ++a) v1[a] = G[0][(size_t)t[0] * rk[0] + a];
      for (int a = 0; a < rk[0]; ++a)
        for (int b = 0; b < rk[1]; ++b) v2[b] += v1[a] * G[1][((size_t)a * n[1] + t[1]) * rk[1] + b];
      for (int b = 0; b < rk[1]; ++b)
        for (int c = 0; c < rk[2]; ++c) v3[c] += v2[b] * G[2][((size_t)b * n[2] + t[2]) * rk[2] + c];
      cxd val = {0, 0};
      for (int c = 0; c < rk[2]; ++c) val += v3[c] * G[3][(size_t)c * n[3] + t[3]];
      const cxd d = val - tval[s];
      e2 += d.re * d.re + d.im * d.im;
    }
    return tnorm > 0 ? std::sqrt(e2 / tnorm) : 0.0;
  };

  int r[3] = {std::min(4, n[0]), 4, std::min(4, n[3])};
  auto cap = [&](int rr[3]) {
    int64_t left = n[0];
    int64_t right = (int64_t)n[1] * n[2] * n[3];
    rr[0] = (int)std::min<int64_t>({(int64_t)rr[0], left, right, (int64_t)rmax});
    left = (int64_t)rr[0] * n[1];
    right = (int64_t)n[2] * n[3];
    rr[1] = (int)std::min<int64_t>({(int64_t)rr[1], left, right, (int64_t)rmax});
    left = (int64_t)rr[1] * n[2];
    right = n[3];
    rr[2] = (int)std::min<int64_t>({(int64_t)rr[2], left, right, (int64_t)rmax});
    // the right-to-left sweep needs r_{k-1} <= n_k r_k
    rr[1] = (int)std::min<int64_t>((int64_t)rr[1], (int64_t)n[2] * rr[2]);
    rr[0] = (int)std::min<int64_t>((int64_t)rr[0], (int64_t)n[1] * rr[1]);
  };
  cap(r);
  // right sets as explicit tuples
  std::vector<std::vector<int>> J[3];   // J[0]: (i2,i3,i4), J[1]: (i3,i4), J[2]: (i4)
  auto random_right = [&](int k) {
    std::vector<int> t;
    for (int q = k + 1; q < 4; ++q) t.push_back((int)(rng() % (uint64_t)n[q]));
    return t;
  };
  auto grow_right = [&]() {
    for (int k = 0; k < 3; ++k) {
      int guard = 0;
      while ((int)J[k].size() < r[k] && guard++ < 100000) {
        std::vector<int> t = random_right(k);
        if (std::find(J[k].begin(), J[k].end(), t) == J[k].end()) J[k].push_back(t);
      }
    }
  };
  grow_right();
  std::vector<std::vector<int>> I[3];   // I[0]: (i1), I[1]: (i1,i2), I[2]: (i1,i2,i3)
  std::vector<cxd> C, Rm, Q;
  double err = 1e300;
  for (int round = 0; round < 40; ++round) {
    for (int sweep = 0; sweep < 2; ++sweep) {
      // left to right
      std::vector<std::vector<int>> left0(1);
      const std::vector<std::vector<int>>* left = &left0;
      for (int k = 0; k < 3; ++k) {
        fibre(f, *left, n[k], k, J[k], C);
        int m = (int)left->size() * n[k];
        int rk = (int)J[k].size();
        Q = C;
        qr_mgs2(Q, m, rk, Rm);
        std::vector<int> rows = maxvol(Q, m, rk);
        I[k].clear();
        for (int row : rows) {
          std::vector<int> t = (*left)[row / n[k]];
          t.push_back(row % n[k]);
          I[k].push_back(t);
        }
        left = &I[k];
      }
      // right to left: k = 3 (last index), then 2, 1
      {
        std::vector<std::vector<int>> right0(1);
        const std::vector<std::vector<int>>* right = &right0;
        for (int k = 3; k >= 1; --k) {
          // fibre A(I[k-1], i_k, right) with rows (a, i) -> use transpose: columns a
          fibre(f, I[k - 1], n[k], k, *right, C);
          int ra = (int)I[k - 1].size(), rb = (int)right->size();
          int m = n[k] * rb;
          std::vector<cxd> T((size_t)m * ra);
          for (int a = 0; a < ra; ++a)
            for (int i = 0; i < n[k]; ++i)
              for (int b = 0; b < rb; ++b) T[(size_t)(i * rb + b) * ra + a] = C[((size_t)a * n[k] + i) * rb + b];
          qr_mgs2(T, m, ra, Rm);
          std::vector<int> rows = maxvol(T, m, ra);
          J[k - 1].clear();
          for (int row : rows) {
            std::vector<int> t;
            t.push_back(row / rb);
            for (int v : (*right)[row % rb]) t.push_back(v);
            J[k - 1].push_back(t);
          }
          right = &J[k - 1];
        }
      }
    }
    // cores from the final left-to-right pass; an unfolding whose fibre matrix already has a
    // numerically dependent column (sigma_min / sigma_max below tol / 4) keeps its rank
    bool saturated[3] = {false, false, false};
    std::vector<std::vector<int>> left0(1);
    const std::vector<std::vector<int>>* left = &left0;
    for (int k = 0; k < 3; ++k) {
      fibre(f, *left, n[k], k, J[k], C);
      int m = (int)left->size() * n[k];
      int rk = (int)J[k].size();
      saturated[k] = sv_ratio(C, m, rk) < 0.25 * tol;
      Q = C;
      qr_mgs2(Q, m, rk, Rm);
      std::vector<int> rows = maxvol(Q, m, rk);
      I[k].clear();
      for (int row : rows) {
        std::vector<int> t = (*left)[row / n[k]];
        t.push_back(row % n[k]);
        I[k].push_back(t);
      }
      // G_k = Q Q[rows]^{-1}: solve Q[rows]^T X^T = Q^T
      std::vector<cxd> S((size_t)rk * rk), B((size_t)rk * m);
      for (int a = 0; a < rk; ++a)
        for (int b = 0; b < rk; ++b) S[(size_t)a * rk + b] = Q[(size_t)rows[b] * rk + a];
      for (int a = 0; a < rk; ++a)
        for (int i = 0; i < m; ++i) B[(size_t)a * m + i] = Q[(size_t)i * rk + a];
      if (!lu_solve(S, rk, B, m)) throw Error(VSIE_E_BREAKDOWN, "TT-cross: singular cross submatrix");
      cores[k].assign((size_t)m * rk, cxd{0, 0});
      for (int i = 0; i < m; ++i)
        for (int a = 0; a < rk; ++a) cores[k][(size_t)i * rk + a] = B[(size_t)a * m + i];
      left = &I[k];
    }
    {
      std::vector<std::vector<int>> right0(1);
      fibre(f, I[2], n[3], 3, right0, C);
      cores[3] = C;   // [a][i4]
    }
    for (int k = 0; k < 3; ++k) ranks[k] = (int)J[k].size();
    err = held_out(cores, ranks);
    if (err <= tol) break;
    int old[3] = {r[0], r[1], r[2]};
    const bool all_sat = saturated[0] && saturated[1] && saturated[2];
    for (int k = 0; k < 3; ++k)
      if (!saturated[k] || all_sat) r[k] = r[k] + std::max(2, r[k] / 2);
    cap(r);
    if (r[0] == old[0] && r[1] == old[1] && r[2] == old[2]) break;   // rank cap reached
    grow_right();
  }
  // TT rounding: the cross overshoots the ranks the accuracy needs (its ranks grow in steps, and
  // interpolation is not an optimal truncation); a rounding with the error budget left by the cross
  // (the two errors combined in quadrature) brings them to near the quasi-optimal TT-SVD ranks.
  // The held-out error is measured again; a rounding that exceeds tol is retried with half the
  // budget, then dropped.
  if (err < tol) {
    double delta = std::sqrt(tol * tol - err * err);
    for (int attempt = 0; attempt < 3; ++attempt, delta *= 0.5) {
      std::vector<cxd> rc[4] = {cores[0], cores[1], cores[2], cores[3]};
      int rr[3] = {ranks[0], ranks[1], ranks[2]};
      tt_round(n, rc, rr, delta);
      const double e = held_out(rc, rr);
      if (e <= tol) {
        for (int k = 0; k < 4; ++k) cores[k].swap(rc[k]);
        for (int k = 0; k < 3; ++k) ranks[k] = rr[k];
        err = e;
        break;
      }
    }
  }
  *err_est = err;
}

}  // namespace vsie
