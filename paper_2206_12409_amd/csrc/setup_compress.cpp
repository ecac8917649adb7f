// TT-cross of a 4D tensor given by an entry function (paper Sec. II-D, Sec. III eq. (14)).
//
// Interpolative TT construction from sampled fibres: nested left index sets I_k (multi-indices
// over i_1..i_k) and right index sets J_k (over i_{k+1}..i_4) are refined by alternating sweeps;
// at every step the fibre matrix C_k = A(I_{k-1}, i_k, J_k) is orthogonalised (QR) and its
// maximum-volume rows give the next index set. Cores follow from the cross interpolation
// formula G_k = Q_k Q_k[rows]^{-1}, G_4 = A(I_3, i_4). Ranks grow (with random enrichment of the
// index sets) until the relative error measured on random held-out entries is below the
// tolerance or the rank cap is reached. The paper uses the two-site DMRG variant of TT-cross;
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
    // cores from the final left-to-right pass
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
    for (int k = 0; k < 3; ++k) r[k] = r[k] + std::max(2, r[k] / 2);
    cap(r);
    if (r[0] == old[0] && r[1] == old[1] && r[2] == old[2]) break;   // rank cap reached
    grow_right();
  }
  *err_est = err;
}

}  // namespace vsie
