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

}  // namespace

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
    // held-out error
    double e2 = 0;
    for (int s = 0; s < ntest; ++s) {
      const int* t = &tidx[4 * s];
      std::vector<cxd> v1(ranks[0]), v2(ranks[1]), v3(ranks[2]);
      for (int a = 0; a < ranks[0]; ++a) v1[a] = cores[0][(size_t)t[0] * ranks[0] + a];
      for (int b = 0; b < ranks[1]; ++b) {
        cxd acc = {0, 0};
        for (int a = 0; a < ranks[0]; ++a) acc += v1[a] * cores[1][((size_t)a * n[1] + t[1]) * ranks[1] + b];
        v2[b] = acc;
      }
      for (int c = 0; c < ranks[2]; ++c) {
        cxd acc = {0, 0};
        for (int b = 0; b < ranks[1]; ++b) acc += v2[b] * cores[2][((size_t)b * n[2] + t[2]) * ranks[2] + c];
        v3[c] = acc;
      }
      cxd val = {0, 0};
      for (int c = 0; c < ranks[2]; ++c) val += v3[c] * cores[3][(size_t)c * n[3] + t[3]];
      cxd d = val - tval[s];
      e2 += d.re * d.re + d.im * d.im;
    }
    err = tnorm > 0 ? sqrt(e2 / tnorm) : 0.0;
    if (err <= tol) break;
    int old[3] = {r[0], r[1], r[2]};
    const bool all_sat = saturated[0] && saturated[1] && saturated[2];
    for (int k = 0; k < 3; ++k)
      if (!saturated[k] || all_sat) r[k] = r[k] + std::max(2, r[k] / 2);
    cap(r);
    if (r[0] == old[0] && r[1] == old[1] && r[2] == old[2]) break;   // rank cap reached
    grow_right();
  }
  *err_est = err;
}

}  // namespace vsie
