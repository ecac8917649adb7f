// C ABI of the hybrid VSIE library: setup orchestration, matrix-vector product and GMRES drivers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <random>
#include <string>

#include "cnn.h"
#include "dense_lu.h"
#include "kernels.h"

using namespace vsie;

struct vsie_handle {
  Handle H;
};

struct vsie_graph {
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
};

struct vsie_net {
  NetState S;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <typename F> int guarded(F&& f) {
  try {
    f();
    return VSIE_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(VSIE_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(VSIE_E_ARG, e.what());
  }
}

template <typename T> T* upload(Handle& H, const std::vector<T>& v) {
  T* d = H.dalloc<T>((int64_t)v.size());
  if (!v.empty()) VSIE_HIP(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return d;
}

template <typename T> std::vector<T> download(const T* d, int64_t n) {
  std::vector<T> v((size_t)std::max<int64_t>(n, 0));
  if (n > 0) VSIE_HIP(hipMemcpy(v.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost));
  return v;
}

template <typename R> cx<R>* upload_cx(Handle& H, const std::vector<cxd>& v) {
  std::vector<cx<R>> c(v.size());
  for (size_t i = 0; i < v.size(); ++i) c[i] = cx<R>{(R)v[i].re, (R)v[i].im};
  return upload(H, c);
}

GridDims grid_dims(const Handle& H) {
  GridDims g;
  g.n1 = H.n[0];
  g.n2 = H.n[1];
  g.n3 = H.n[2];
  g.ne1 = H.ne[0];
  g.ne2 = H.ne[1];
  g.ne3 = H.ne[2];
  g.ob1 = H.ob[0];
  g.ob2 = H.ob[1];
  g.ob3 = H.ob[2];
  g.nv = H.nv;
  g.Ne = H.Ne;
  return g;
}

RwgDev make_rwg_dev(Handle& H, const Rwg& R) {
  RwgDev d{};
  d.m = R.m;
  if (R.m == 0) return d;
  d.verts = upload(H, R.verts);
  d.tris = upload(H, R.tris);
  d.area = upload(H, R.area);
  std::vector<int> tpm(2 * R.m), flpm(2 * R.m), fpm(2 * R.m);
  for (int i = 0; i < R.m; ++i) {
    tpm[2 * i] = R.tp[i];
    tpm[2 * i + 1] = R.tm[i];
    flpm[2 * i] = R.flp[i];
    flpm[2 * i + 1] = R.flm[i];
    fpm[2 * i] = R.fp[i];
    fpm[2 * i + 1] = R.fm[i];
  }
  d.tpm = upload(H, tpm);
  d.flpm = upload(H, flpm);
  d.fpm = upload(H, fpm);
  d.len = upload(H, R.len);
  return d;
}

template <typename R> cx<R>* twiddles(Handle& H, int L) {
  std::vector<cxd> t(L);
  for (int m = 0; m < L; ++m) {
    long double a = -2.0L * 3.14159265358979323846264338327950288L * m / L;
    t[m] = cxd{(double)cosl(a), (double)sinl(a)};
  }
  return upload_cx<R>(H, t);
}

// ---------------------------------------------------------------------------------------------
// volume convolution data: generator on the extended-grid octant, circulant spectra
void setup_volume(Handle& H) {
  hipStream_t st = H.stream;
  for (int v = 0; v < 2; ++v) {
    const std::vector<int> ord = zconv_order(H.P[2], H.P[0], H.P[1], v == 0, 0);
    if (!ord.empty()) H.d_zorder[v] = upload<int>(H, ord);
  }
  GaussTab gt_h;
  fill_gauss_table(&gt_h);
  GaussTab* gt = H.dalloc<GaussTab>(1);
  VSIE_HIP(hipMemcpy(gt, &gt_h, sizeof(GaussTab), hipMemcpyHostToDevice));
  CellRule cr;
  cr.n_duffy = 14;
  cr.digits = 18.0;
  cr.n_min = 4;
  cr.n_max = 18;
  H.d_oct = H.dalloc<cxd>(6 * H.Ne);
  launch_generator(st, gt, H.ne, H.k0 * H.h, cr, H.d_oct);
  VSIE_HIP(hipGetLastError());
  const int64_t PT = (int64_t)H.P[0] * H.P[1] * H.P[2];
  cxd* full = nullptr;
  VSIE_HIP(hipMalloc(&full, sizeof(cxd) * 6 * PT));
  cxd* full2 = nullptr;
  if (hipMalloc(&full2, sizeof(cxd) * 6 * PT) != hipSuccess) {
    (void)hipFree(full);
    throw Error(VSIE_E_NOMEM, "generator spectra workspace");
  }
  cxd* tw[3];
  for (int a = 0; a < 3; ++a) tw[a] = twiddles<double>(H, H.P[a]);
  launch_embed_circulant(st, H.d_oct, H.ne, H.P, full);
  // full forward 3D FFT of the 6 components: x (rows), y (strided), z (strided)
  const int P1 = H.P[0], P2 = H.P[1], P3 = H.P[2];
  fft_rows<double>(st, P1, true, full, full2, P1, P1, P1, P1, 6LL * P2 * P3, tw[0]);
  fft_strided<double>(st, P2, true, full2, full, P2, P2, P1, P1, P1, 6LL * P3, (int64_t)P2 * P1, (int64_t)P2 * P1, tw[1]);
  fft_strided<double>(st, P3, true, full, full2, P3, P3, (int64_t)P1 * P2, (int64_t)P1 * P2, P1 * P2, 6,
                      (int64_t)P1 * P2 * P3, (int64_t)P1 * P2 * P3, tw[2]);
  VSIE_HIP(hipGetLastError());
  const int64_t SO = (int64_t)(P1 / 2 + 1) * (P2 / 2 + 1) * (P3 / 2 + 1);
  const double scale = H.h * H.h * H.h / ((double)P1 * P2 * P3);
  H.d64.spec = H.dalloc<cxd>(6 * SO);
  launch_extract_octant<double>(st, full2, H.P, scale, H.d64.spec);
  if (H.opts.precision) {
    H.d32.spec = H.dalloc<cxf>(6 * SO);
    launch_extract_octant<float>(st, full2, H.P, scale, H.d32.spec);
  }
  VSIE_HIP(hipStreamSynchronize(st));
  (void)hipFree(full);
  (void)hipFree(full2);
  for (int a = 0; a < 3; ++a) {
    H.d64.tw[a] = tw[a];
    if (H.opts.precision) H.d32.tw[a] = twiddles<float>(H, H.P[a]);
  }
  // body diagonal and mask
  std::vector<cxd> dv(H.nv, cxd{0, 0});
  std::vector<uint8_t> mask(H.nv, 0);
  const double h3 = H.h * H.h * H.h;
  for (int p = 0; p < H.nv; ++p)
    if (H.chi[p].re != 0 || H.chi[p].im != 0) {
      dv[p] = h3 * cinv(H.chi[p]);
      mask[p] = 1;
    }
  H.d_mask = upload(H, mask);
  // tissue run [lo, hi) of each x row; ~lo marks a run with air inside it
  std::vector<int2> runs((size_t)H.n[1] * H.n[2], int2{0, 0});
  for (size_t r = 0; r < runs.size(); ++r) {
    const uint8_t* m = mask.data() + r * H.n[0];
    int lo = -1, hi = 0, cnt = 0;
    for (int i = 0; i < H.n[0]; ++i)
      if (m[i]) {
        if (lo < 0) lo = i;
        hi = i + 1;
        ++cnt;
      }
    if (cnt > 0) runs[r] = int2{cnt == hi - lo ? lo : ~lo, hi};
  }
  H.d_runs = upload(H, runs);
  H.d64.dv_chi = upload_cx<double>(H, dv);
  if (H.opts.precision) H.d32.dv_chi = upload_cx<float>(H, dv);
}

// ---------------------------------------------------------------------------------------------
// pFFT: grid CSR of the projection, device weights, precorrection of near pairs
void setup_pfft(Handle& H) {
  hipStream_t st = H.stream;
  const int mn = H.mn;
  std::vector<int> base_ext(3 * mn);
  for (int i = 0; i < mn; ++i)
    for (int a = 0; a < 3; ++a) base_ext[3 * i + a] = H.base[3 * i + a] + H.ob[a];
  H.d_base = upload(H, base_ext);
  H.d64.W = upload(H, H.Wh);
  if (H.opts.precision) {
    std::vector<float> wf(H.Wh.begin(), H.Wh.end());
    H.d32.W = upload(H, wf);
  }
  // grid CSR by extended-grid voxel (entries sorted by voxel, then RWG)
  struct Ent {
    int64_t v;
    int n;
    int j;
  };
  std::vector<Ent> ents;
  ents.reserve((size_t)mn * 125);
  for (int n = 0; n < mn; ++n)
    for (int j = 0; j < 125; ++j) {
      int j1 = j % 5, j2 = (j / 5) % 5, j3 = j / 25;
      int64_t v = (base_ext[3 * n] + j1) + (int64_t)H.ne[0] * ((base_ext[3 * n + 1] + j2) + (int64_t)H.ne[1] * (base_ext[3 * n + 2] + j3));
      ents.push_back({v, n, j});
    }
  std::sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) { return a.v != b.v ? a.v < b.v : a.n < b.n; });
  std::vector<int> vox2row(H.Ne, -1), rowptr, rowrwg;
  std::vector<double> roww;
  for (size_t e = 0; e < ents.size(); ++e) {
    if (e == 0 || ents[e].v != ents[e - 1].v) {
      vox2row[ents[e].v] = (int)rowptr.size();
      rowptr.push_back((int)e);
    }
    rowrwg.push_back(ents[e].n);
    for (int a = 0; a < 3; ++a) roww.push_back(H.Wh[(size_t)ents[e].n * 375 + a * 125 + ents[e].j]);
  }
  rowptr.push_back((int)ents.size());
  H.n_gridrows = (int)rowptr.size() - 1;
  H.nnz_grid = (int64_t)ents.size();
  // per x row (i2, i3) of the extended grid: does any of its voxels carry a projection row
  std::vector<uint8_t> rowhas((size_t)H.ne[1] * H.ne[2], 0);
  for (size_t e = 0; e < ents.size(); ++e) rowhas[(size_t)(ents[e].v / H.ne[0])] = 1;
  H.d_rowhasproj = upload(H, rowhas);
  H.d_vox2row = upload(H, vox2row);
  H.d_rowptr = upload(H, rowptr);
  H.d_rowrwg = upload(H, rowrwg);
  H.d64.roww = upload(H, roww);
  if (H.opts.precision) {
    std::vector<float> rf(roww.begin(), roww.end());
    H.d32.roww = upload(H, rf);
  }

  // --- precorrection pairs
  const int D = H.opts.precorrect_dist;
  std::vector<int> pm, pn;
  for (int m = 0; m < mn; ++m)
    for (int n = 0; n < mn; ++n) {
      int gap = 0;
      for (int a = 0; a < 3; ++a) {
        int bm = H.base[3 * m + a], bn = H.base[3 * n + a];
        int g = std::max({bn - (bm + 4), bm - (bn + 4), 0});
        gap = std::max(gap, g);
      }
      if (gap <= D) {
        pm.push_back(m);
        pn.push_back(n);
      }
    }
  std::vector<int> vp, vn, vox;   // tissue voxel (flat body index), RWG, ext coords
  std::vector<double> vc;
  for (int n = 0; n < mn; ++n) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::max(0, H.base[3 * n + a] - D);
      hi[a] = std::min(H.n[a] - 1, H.base[3 * n + a] + 4 + D);
    }
    for (int i3 = lo[2]; i3 <= hi[2]; ++i3)
      for (int i2 = lo[1]; i2 <= hi[1]; ++i2)
        for (int i1 = lo[0]; i1 <= hi[0]; ++i1) {
          int p = i1 + H.n[0] * (i2 + H.n[1] * i3);
          if (H.chi[p].re == 0 && H.chi[p].im == 0) continue;
          vp.push_back(p);
          vn.push_back(n);
          vox.push_back(i1 + H.ob[0]);
          vox.push_back(i2 + H.ob[1]);
          vox.push_back(i3 + H.ob[2]);
          vc.push_back(H.origin[0] + (i1 + 0.5) * H.h);
          vc.push_back(H.origin[1] + (i2 + 0.5) * H.h);
          vc.push_back(H.origin[2] + (i3 + 0.5) * H.h);
        }
  }
  const int64_t nnp = (int64_t)pm.size(), nvp = (int64_t)vp.size();
  int* d_pm = H.dalloc<int>(nnp);
  int* d_pn = H.dalloc<int>(nnp);
  VSIE_HIP(hipMemcpy(d_pm, pm.data(), sizeof(int) * nnp, hipMemcpyHostToDevice));
  VSIE_HIP(hipMemcpy(d_pn, pn.data(), sizeof(int) * nnp, hipMemcpyHostToDevice));
  cxd* d_direct = H.dalloc<cxd>(nnp);
  cxd* d_grid = H.dalloc<cxd>(nnp);
  launch_zcc_pairs(st, H.dnear, H.dnear, d_pm, d_pn, nnp, H.k0, d_direct);
  launch_pfft_wtw(st, H.d64.W, H.d_base, H.d_oct, H.ne, d_pm, d_pn, nnp, d_grid);
  std::vector<cxd> vdir, vgrid;
  if (nvp > 0) {
    int* d_vn = upload(H, vn);
    int* d_vox = upload(H, vox);
    double* d_vc = upload(H, vc);
    cxd* d_vdir = H.dalloc<cxd>(3 * nvp);
    cxd* d_vgrid = H.dalloc<cxd>(3 * nvp);
    launch_zbc_near(st, H.dnear, d_vc, d_vn, nvp, H.h, H.k0, d_vdir);
    launch_pfft_tw_voxels(st, H.d64.W, H.d_base, H.d_oct, H.ne, d_vox, d_vn, nvp, d_vgrid);
    VSIE_HIP(hipStreamSynchronize(st));
    vdir = download(d_vdir, 3 * nvp);
    vgrid = download(d_vgrid, 3 * nvp);
  }
  VSIE_HIP(hipGetLastError());
  VSIE_HIP(hipStreamSynchronize(st));
  std::vector<cxd> ndir = download(d_direct, nnp), ngrid = download(d_grid, nnp);
  const double h3 = H.h * H.h * H.h;
  struct Coo {
    int64_t r, c;
    cxd v;
  };
  std::vector<Coo> coo;
  coo.reserve(nnp + 6 * nvp);
  const int64_t offn = H.mf, offb = (int64_t)H.mf + H.mn;
  for (int64_t e = 0; e < nnp; ++e) coo.push_back({offn + pm[e], offn + pn[e], ndir[e] - h3 * ngrid[e]});
  for (int64_t e = 0; e < nvp; ++e)
    for (int a = 0; a < 3; ++a) {
      cxd v = vdir[3 * e + a] - h3 * vgrid[3 * e + a];
      int64_t rb = offb + (int64_t)a * H.nv + vp[e];
      coo.push_back({rb, offn + vn[e], v});
      coo.push_back({offn + vn[e], rb, v});
    }
  std::sort(coo.begin(), coo.end(), [](const Coo& a, const Coo& b) { return a.r != b.r ? a.r < b.r : a.c < b.c; });
  std::vector<int> rowid, rp, col;
  std::vector<cxd> val;
  for (size_t e = 0; e < coo.size(); ++e) {
    if (e == 0 || coo[e].r != coo[e - 1].r) {
      rowid.push_back((int)coo[e].r);
      rp.push_back((int)col.size());
    }
    if (!col.empty() && e > 0 && coo[e].r == coo[e - 1].r && coo[e].c == coo[e - 1].c) {
      val.back() += coo[e].v;
      continue;
    }
    col.push_back((int)coo[e].c);
    val.push_back(coo[e].v);
  }
  rp.push_back((int)col.size());
  H.n_pcrows = (int)rowid.size();
  H.pc_nnz = (int64_t)col.size();
  H.d_pc_rowid = upload(H, rowid);
  H.d_pc_rowptr = upload(H, rp);
  H.d_pc_col = upload(H, col);
  H.d64.pc_val = upload_cx<double>(H, val);
  if (H.opts.precision) H.d32.pc_val = upload_cx<float>(H, val);
}

// ---------------------------------------------------------------------------------------------
// far conductors: dense block, ACA of the near-far block, TT-cross of the far coupling
// dense far block (eq. (6)), symmetric: only the upper-triangle tiles are assembled and stored
template <typename T> static T* share_alloc(int64_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess)
    throw Error(VSIE_E_NOMEM, "hipMalloc of the dense far block failed");
  return (T*)p;
}

// assembled once per set of far conductors (H.far_share set beforehand: adopted from the operator
// it was shared with)
void setup_dense_far(Handle& H) {
  const int T = (H.mf + SYM_TB - 1) / SYM_TB;
  H.sym_T = T;
  const int64_t nt = (int64_t)T * (T + 1) / 2;
  const int64_t per = (int64_t)SYM_TB * SYM_TB;
  if (!H.far_share) {
    auto sh = std::make_shared<FarShare>();
    std::vector<int> tiles;
    for (int I = 0; I < T; ++I)
      for (int J = I; J < T; ++J) {
        tiles.push_back(I);
        tiles.push_back(J);
      }
    sh->T = T;
    sh->k0 = H.k0;
    sh->verts = H.far.verts;
    sh->tris = H.far.tris;
    sh->ea = H.far.ea;
    sh->eb = H.far.eb;
    sh->tp = H.far.tp;
    sh->tm = H.far.tm;
    sh->tiles = share_alloc<int>((int64_t)tiles.size());
    VSIE_HIP(hipMemcpy(sh->tiles, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice));
    sh->z64 = share_alloc<cxd>(nt * per);
    const int64_t chunk = std::max<int64_t>(1, (1LL << 26) / per);
    for (int64_t t0 = 0; t0 < nt; t0 += chunk)
      launch_zcc_packed(H.stream, H.dfar, H.k0, sh->tiles, t0, std::min(chunk, nt - t0), sh->z64 + t0 * per);
    VSIE_HIP(hipGetLastError());
    VSIE_HIP(hipStreamSynchronize(H.stream));
    H.device_bytes += sizeof(cxd) * nt * per;
    H.far_share = sh;
  }
  H.d_tiles = H.far_share->tiles;
  H.d64.Zff = H.far_share->z64;
  H.d64.sym_part = H.dalloc<cxd>(nt * 2 * SYM_TB);
}

void copy_zff_c64(Handle& H) {
  const int64_t T = H.sym_T;
  const int64_t n = T * (T + 1) / 2 * SYM_TB * SYM_TB;
  FarShare& sh = *H.far_share;
  if (!sh.z32) {
    sh.z32 = share_alloc<cxf>(n);
    launch_d2f(H.stream, sh.z64, sh.z32, n);
    VSIE_HIP(hipStreamSynchronize(H.stream));
    H.device_bytes += sizeof(cxf) * n;
  }
  H.d32.Zff = sh.z32;
  H.d32.sym_part = H.dalloc<cxf>(T * (T + 1) / 2 * 2 * SYM_TB);
}

void setup_aca(Handle& H) {
  // partially pivoted ACA of Z_nf (m_n x m_f) ~ sum_l u_l v_l^T; stored as U V^* (V = conj(v)).
  // The stopping estimate ||u_k|| ||v_k|| <= tol ||S_k||_F only sees the rows the pivots visited;
  // once it holds, the error is measured on held-out rows (exact rows of the block against U V^*)
  // and, while that exceeds tol, the approximation continues from the worst held-out row.
  const int mn = H.mn, mf = H.mf;
  cxd* d_row = H.dalloc<cxd>(mf);
  cxd* d_col = H.dalloc<cxd>(mn);
  std::vector<std::vector<cxd>> us, vs;
  std::vector<char> used_row(mn, 0), used_col(mf, 0);
  int i = 0;
  double norm2 = 0;
  const int kmax = std::min({H.opts.aca_rank_max, mn, mf, 256});
  // held-out rows: a seeded sample of the near RWGs, at most 32
  std::vector<int> hold;
  {
    std::mt19937_64 rng(H.opts.seed * 7919 + 17);
    std::vector<int> all(mn);
    std::iota(all.begin(), all.end(), 0);
    std::shuffle(all.begin(), all.end(), rng);
    all.resize(std::min(mn, 32));
    std::sort(all.begin(), all.end());
    hold = all;
  }
  std::vector<std::vector<cxd>> hold_rows;
  double hold_norm2 = 0;
  for (int q : hold) {
    launch_zcc_dense(H.stream, H.dnear, H.dfar, H.k0, q, 1, d_row);
    hold_rows.push_back(download(d_row, mf));
    for (const cxd& z : hold_rows.back()) hold_norm2 += z.re * z.re + z.im * z.im;
  }
  // relative error of the current U V^T on the held-out rows, and the worst row
  auto held_out = [&](int* worst) {
    double e2 = 0, wbest = -1;
    *worst = -1;
    for (size_t h = 0; h < hold.size(); ++h) {
      double r2 = 0;
      for (int j = 0; j < mf; ++j) {
        cxd d = hold_rows[h][j];
        for (size_t l = 0; l < us.size(); ++l) d -= us[l][hold[h]] * vs[l][j];
        r2 += d.re * d.re + d.im * d.im;
      }
      e2 += r2;
      if (r2 > wbest && !used_row[hold[h]]) { wbest = r2; *worst = hold[h]; }
    }
    return hold_norm2 > 0 ? std::sqrt(e2 / hold_norm2) : 0.0;
  };
  for (int it = 0; it < 4 * kmax && (int)us.size() < kmax; ++it) {
    used_row[i] = 1;
    launch_zcc_dense(H.stream, H.dnear, H.dfar, H.k0, i, 1, d_row);
    std::vector<cxd> r = download(d_row, mf);
    for (size_t l = 0; l < us.size(); ++l)
      for (int j = 0; j < mf; ++j) r[j] -= us[l][i] * vs[l][j];
    int jb = -1;
    double best = 0;
    for (int j = 0; j < mf; ++j) {
      if (used_col[j]) continue;
      double a = r[j].re * r[j].re + r[j].im * r[j].im;
      if (a > best) { best = a; jb = j; }
    }
    if (jb < 0 || best == 0) {
      int nxt = -1;
      for (int q = 0; q < mn; ++q)
        if (!used_row[q]) { nxt = q; break; }
      if (nxt < 0) break;
      i = nxt;
      continue;
    }
    used_col[jb] = 1;
    cxd inv = cinv(r[jb]);
    std::vector<cxd> v(mf);
    for (int j = 0; j < mf; ++j) v[j] = r[j] * inv;
    launch_zcc_dense(H.stream, H.dfar, H.dnear, H.k0, jb, 1, d_col);
    std::vector<cxd> u = download(d_col, mn);
    for (size_t l = 0; l < us.size(); ++l)
      for (int q = 0; q < mn; ++q) u[q] -= vs[l][jb] * us[l][q];
    double nu = 0, nvv = 0;
    for (auto& z : u) nu += z.re * z.re + z.im * z.im;
    for (auto& z : v) nvv += z.re * z.re + z.im * z.im;
    cxd cross = {0, 0};
    for (size_t l = 0; l < us.size(); ++l) {
      cxd a = {0, 0}, b = {0, 0};
      for (int q = 0; q < mn; ++q) a += mul_conj_a(us[l][q], u[q]);
      for (int j = 0; j < mf; ++j) b += mul_conj_a(vs[l][j], v[j]);
      cross += a * b;
    }
    norm2 += 2.0 * cross.re + nu * nvv;
    us.push_back(u);
    vs.push_back(v);
    if (sqrt(nu * nvv) <= H.opts.aca_tol * sqrt(std::max(norm2, 0.0))) {
      int worst = -1;
      if (held_out(&worst) <= H.opts.aca_tol || worst < 0) break;
      i = worst;   // the estimate was optimistic: continue from the worst held-out row
      continue;
    }
    int nxt = -1;
    best = -1;
    for (int q = 0; q < mn; ++q) {
      if (used_row[q]) continue;
      double a = u[q].re * u[q].re + u[q].im * u[q].im;
      if (a > best) { best = a; nxt = q; }
    }
    if (nxt < 0) break;
    i = nxt;
  }
  const int k = (int)us.size();
  H.aca_k = k;
  H.aca_U.assign((size_t)mn * k, cxd{0, 0});
  H.aca_V.assign((size_t)mf * k, cxd{0, 0});
  for (int l = 0; l < k; ++l) {
    for (int q = 0; q < mn; ++q) H.aca_U[(size_t)q * k + l] = us[l][q];
    for (int j = 0; j < mf; ++j) H.aca_V[(size_t)j * k + l] = conj(vs[l][j]);
  }
}

// the host keeps U (m_n x k) and V (m_f x k) row-major; the device holds them rank-major
void upload_aca(Handle& H) {
  if (H.aca_k == 0) return;
  const int k = H.aca_k;
  auto rank_major = [k](const std::vector<cxd>& A) {
    const size_t m = A.size() / k;
    std::vector<cxd> B(A.size());
    for (size_t i = 0; i < m; ++i)
      for (int l = 0; l < k; ++l) B[(size_t)l * m + i] = A[i * k + l];
    return B;
  };
  const std::vector<cxd> Ut = rank_major(H.aca_U), Vt = rank_major(H.aca_V);
  H.d64.U = upload_cx<double>(H, Ut);
  H.d64.V = upload_cx<double>(H, Vt);
  if (H.opts.precision) {
    H.d32.U = upload_cx<float>(H, Ut);
    H.d32.V = upload_cx<float>(H, Vt);
  }
}

// far coupling entry, 1 volume x 1 surface point:
//   Z[chi](i1,i2,i3,n) = -h^3 sum_sides s (l/2) [ D(r_c - c_T) (c_T - p_T) ]_chi
struct FarCoupling : EntryFn {
  const Handle& H;
  int chi;
  std::vector<V3> cen[2], vec[2];
  FarCoupling(const Handle& h, int c) : H(h), chi(c) {
    const Rwg& R = H.far;
    for (int side = 0; side < 2; ++side) {
      cen[side].resize(R.m);
      vec[side].resize(R.m);
      for (int i = 0; i < R.m; ++i) {
        int t = side == 0 ? R.tp[i] : R.tm[i];
        int fv = side == 0 ? R.fp[i] : R.fm[i];
        V3 c = (1.0 / 3.0) * (R.vert(R.tris[3 * t]) + R.vert(R.tris[3 * t + 1]) + R.vert(R.tris[3 * t + 2]));
        double s = side == 0 ? 1.0 : -1.0;
        cen[side][i] = c;
        vec[side][i] = (s * 0.5 * R.len[i]) * (c - R.vert(fv));
      }
    }
  }
  void eval(const std::vector<int>& idx, std::vector<cxd>& out) override {
    const int64_t n = (int64_t)idx.size() / 4;
    out.resize(n);
    const double h3 = H.h * H.h * H.h;
    parallel_for(n, 16, [&](int64_t a, int64_t b) {
      for (int64_t e = a; e < b; ++e) {
        const int* t = &idx[4 * e];
        V3 r = {H.origin[0] + (t[0] + 0.5) * H.h, H.origin[1] + (t[1] + 0.5) * H.h, H.origin[2] + (t[2] + 0.5) * H.h};
        cxd acc = {0, 0};
        for (int side = 0; side < 2; ++side) {
          V3 v = vec[side][t[3]];
          cxd vv[3] = {{v.x, 0}, {v.y, 0}, {v.z, 0}};
          cxd o[3];
          dyad_apply(r - cen[side][t[3]], vv, H.k0, o);
          acc += o[chi];
        }
        out[e] = (-h3) * acc;
      }
    });
  }
};

void setup_tt(Handle& H) {
  const int n4[4] = {H.n[0], H.n[1], H.n[2], H.mf};
  for (int chi = 0; chi < 3; ++chi) {
    FarCoupling f(H, chi);
    int ranks[3];
    double err = 0;
    tt_cross(f, n4, H.opts.tt_tol, H.opts.tt_rank_max, H.opts.seed + 7919ull * chi, H.tt_host[chi], ranks, &err);
    for (int k = 0; k < 3; ++k) H.tt_r[chi][k] = ranks[k];
    H.tt_err[chi] = err;
  }
}

// Device copies of the four cores of one component (eq. (14)).
void upload_tt(Handle& H, int chi) {
  for (int k = 0; k < 4; ++k) {
    H.d64.G[chi][k] = upload_cx<double>(H, H.tt_host[chi][k]);
    if (H.opts.precision) H.d32.G[chi][k] = upload_cx<float>(H, H.tt_host[chi][k]);
  }
}

// Autotuner of the z pass (radix and tile): every compiled candidate for this FFT length runs on
// the operator's own work buffer and spectra (three timed launches after one warm-up), and the
// fastest is kept with its block order.
template <typename R> static void tune_zpass(Handle& H, OpData<R>& D) {
  const int L = H.P[2];
  const bool f64 = sizeof(R) == 8;
  const int v = f64 ? 0 : 1;
  if (L < 64 || L > 1024) return;
  hipStream_t st = H.stream;
  const int P1 = H.P[0], P2 = H.P[1], ne3 = H.ne[2];
  VSIE_HIP(hipMemsetAsync(D.bufC, 0, sizeof(cx<R>) * 3 * (size_t)ne3 * P2 * P1, st));
  hipEvent_t e0, e1;
  VSIE_HIP(hipEventCreate(&e0));
  VSIE_HIP(hipEventCreate(&e1));
  double best = 1e300;
  int bc = 0;
  int* orders[3] = {};
  for (int c = 0; c < 3; ++c) {
    H.ztime[v][c] = 0;
    if (!zconv_candidate(L, f64, c)) continue;
    orders[c] = upload<int>(H, zconv_order(L, P1, P2, f64, c));
    fft_z_conv<R>(st, L, D.bufC, ne3, P1, P2, D.spec, D.tw[2], orders[c], c);
    VSIE_HIP(hipEventRecord(e0, st));
    for (int k = 0; k < 3; ++k) fft_z_conv<R>(st, L, D.bufC, ne3, P1, P2, D.spec, D.tw[2], orders[c], c);
    VSIE_HIP(hipEventRecord(e1, st));
    VSIE_HIP(hipEventSynchronize(e1));
    float ms = 0;
    VSIE_HIP(hipEventElapsedTime(&ms, e0, e1));
    H.ztime[v][c] = ms / 3.0;
    if (ms / 3.0 < best) {
      best = ms / 3.0;
      bc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  H.zcand[v] = bc;
  H.d_zorder[v] = orders[bc];
}

template <typename R> void alloc_work(Handle& H, OpData<R>& D) {
  D.gridA = H.dalloc<cx<R>>(3 * H.Ne);
  D.bufB = H.dalloc<cx<R>>(3LL * H.ne[2] * H.ne[1] * H.P[0]);
  D.bufC = H.dalloc<cx<R>>(3LL * H.ne[2] * H.P[1] * H.P[0]);
  D.tt_work = H.dalloc<cx<R>>(tt_work_elems(H.n, std::max(H.mf, 1)));
  D.small_work = H.dalloc<cx<R>>(512 * 256 + 512);
  if (H.n_gridrows > 0) D.projv = H.dalloc<cx<R>>(3LL * H.n_gridrows);
  if (H.mf > 0) D.dual_part = H.dalloc<cx<R>>(lr_dual_part_elems(H.mf));
}

// ---------------------------------------------------------------------------------------------
const char* const kStageNames[Handle::NSTAGE] = {
    "build_grid", "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv",       "fft_x_inv", "body_out",
    "pfft_gather", "gemv_far", "precorrect", "aca",       "tt_pre",    "gemv_far_reduce", "tt_post"};

// Accumulate the stage times of every pending product (waits for their events).
static void drain_profile(Handle& H) {
  for (int k = H.ring_count; k > 0; --k) {
    const int slot = (H.ring_head - k + Handle::PROF_RING) % Handle::PROF_RING;
    for (int s = 0; s < Handle::NSTAGE; ++s)
      if (H.ev_mask[slot] & (1u << s)) {
        VSIE_HIP(hipEventSynchronize(H.ev[slot][2 * s + 1]));
        float ms = 0;
        VSIE_HIP(hipEventElapsedTime(&ms, H.ev[slot][2 * s], H.ev[slot][2 * s + 1]));
        H.prof_ms[s] += ms;
        H.prof_calls[s] += 1;
      }
  }
  H.ring_count = 0;
}

// Per-stage HIP events of one product, recorded on the stream the stage runs on.
struct StageTimer {
  Handle& H;
  hipStream_t st;
  int slot = -1;
  StageTimer(Handle& h, hipStream_t s) : H(h), st(s) {
    if (!H.prof) return;
    if (H.ring_count == Handle::PROF_RING) drain_profile(H);
    slot = H.ring_head;
    H.ev_mask[slot] = 0;
  }
  void begin(int s, hipStream_t on = nullptr) {
    if (slot < 0 || !(H.prof_stages & (1u << s))) return;
    VSIE_HIP(hipEventRecord(H.ev[slot][2 * s], on ? on : st));
    H.ev_mask[slot] |= 1u << s;
  }
  void end(int s, hipStream_t on = nullptr) {
    if (slot >= 0 && (H.prof_stages & (1u << s))) VSIE_HIP(hipEventRecord(H.ev[slot][2 * s + 1], on ? on : st));
  }
  void collect() {
    if (slot < 0) return;
    H.ring_head = (slot + 1) % Handle::PROF_RING;
    ++H.ring_count;
  }
};

// One product (eq. (15)). The dense far block only reads x_f and writes y_f, so it runs on a
// second stream (default priority, forked from and joined back into the caller's stream by
// events) concurrently with the volume convolution and pFFT chain; everything that accumulates
// into y_f, y_n or y_b after both runs on the caller's stream.
static void make_streams(Handle& H) {
  VSIE_HIP(hipStreamCreateWithFlags(&H.side, hipStreamNonBlocking));
  VSIE_HIP(hipEventCreateWithFlags(&H.fork, hipEventDisableTiming));
  VSIE_HIP(hipEventCreateWithFlags(&H.join, hipEventDisableTiming));
}

static BodyMask body_mask(const Handle& H) { return BodyMask{H.d_mask, H.d_runs}; }

// Volume convolution with the pFFT projection and interpolation of the near currents
// (Sec. II-B, eq. (13)): y_b and y_n from x_b and x_n (x_n null when there are no near currents).
template <typename R>
static void volume_chain(Handle& H, OpData<R>& D, const cx<R>* xn, const cx<R>* xb, cx<R>* yn, cx<R>* yb,
                         hipStream_t st, StageTimer& T) {
  GridDims g = grid_dims(H);
  const int mn = H.mn;
  const int P1 = H.P[0], P2 = H.P[1], P3 = H.P[2];
  const int ne1 = H.ne[0], ne2 = H.ne[1], ne3 = H.ne[2];
  // the grid build (stage 0) is fused into the first FFT pass (stage 1)
  T.begin(1, st);
  fft_rows_grid<R>(st, P1, xb, mn ? xn : nullptr, body_mask(H), mn ? H.d_vox2row : nullptr, H.d_rowhasproj, H.d_rowptr,
                   H.d_rowrwg, D.roww, H.n_gridrows, D.projv, g, D.bufB, D.tw[0]);
  T.end(1, st);
  T.begin(2, st);
  fft_strided<R>(st, P2, true, D.bufB, D.bufC, ne2, P2, P1, P1, P1, 3LL * ne3, (int64_t)ne2 * P1, (int64_t)P2 * P1, D.tw[1]);
  T.end(2, st);
  T.begin(3, st);
  fft_z_conv<R>(st, P3, D.bufC, ne3, P1, P2, D.spec, D.tw[2], H.d_zorder[sizeof(R) == 8 ? 0 : 1],
                H.zcand[sizeof(R) == 8 ? 0 : 1]);
  T.end(3, st);
  T.begin(4, st);
  fft_strided<R>(st, P2, false, D.bufC, D.bufB, P2, ne2, P1, P1, P1, 3LL * ne3, (int64_t)P2 * P1, (int64_t)ne2 * P1, D.tw[1]);
  T.end(4, st);
  T.begin(5, st);
  fft_rows<R>(st, P1, false, D.bufB, D.gridA, P1, ne1, P1, ne1, 3LL * ne3 * ne2, D.tw[0]);
  T.end(5, st);
  T.begin(6, st);
  launch_body_out<R>(st, xb, D.gridA, D.dv_chi, H.d_mask, yb, g);
  T.end(6, st);
  if (mn) {
    T.begin(7, st);
    launch_pfft_gather<R>(st, D.W, H.d_base, D.gridA, yn, mn, g);
    T.end(7, st);
  }
}

template <typename R> static bool tt_desc(const Handle& H, const OpData<R>& D, TTDesc<R>& td, int r3[3]) {
  bool have = H.mf > 0;
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 4; ++k) have = have && D.G[c][k] != nullptr;
  for (int c = 0; c < 3; ++c) {
    td.G1[c] = D.G[c][0];
    td.G2[c] = D.G[c][1];
    td.G3[c] = D.G[c][2];
    td.G4[c] = D.G[c][3];
    td.r1[c] = have ? H.tt_r[c][0] : 0;
    td.r2[c] = have ? H.tt_r[c][1] : 0;
    td.r3[c] = have ? H.tt_r[c][2] : 0;
    r3[c] = td.r3[c];
  }
  return have;
}

// far_done: y_f already holds Z_ff x_f (the batched tile pass of vsie_matvec)
template <typename R>
void matvec_one(Handle& H, OpData<R>& D, const cx<R>* x, cx<R>* y, hipStream_t st, bool far_done = false) {
  if (H.concurrent && !H.side) make_streams(H);
  // far-block chain: the second stream when concurrent, else the caller's stream after the
  // volume chain
  const bool conc = H.concurrent && H.mf;
  hipStream_t fs = conc ? H.side : st;
  StageTimer T(H, st);
  const int mf = H.mf, mn = H.mn;
  const cx<R>* xf = x;
  const cx<R>* xn = x + mf;
  const cx<R>* xb = x + mf + mn;
  cx<R>* yf = y;
  cx<R>* yn = y + mf;
  cx<R>* yb = y + mf + mn;
  TTDesc<R> td;
  int r3[3];
  const bool have_tt = tt_desc(H, D, td, r3);
  // dense far block (writes y_f), then the TT coupling's x-side work and its y_f part
  auto far_chain = [&]() {
    if (!far_done) {
      T.begin(8, fs);
      launch_symv_tiles<R>(fs, D.Zff, H.d_tiles, H.sym_T, xf, mf, D.sym_part);
      T.end(8, fs);
      T.begin(12, fs);
      launch_symv_reduce<R>(fs, D.sym_part, H.sym_T, mf, yf);
      T.end(12, fs);
    }
    if (have_tt) {
      T.begin(11, fs);
      launch_tt_pre<R>(fs, td, H.n, mf, xf, xb, body_mask(H), yf, D.tt_work);
      T.end(11, fs);
    }
  };
  if (conc) {
    VSIE_HIP(hipEventRecord(H.fork, st));
    VSIE_HIP(hipStreamWaitEvent(H.side, H.fork, 0));
    far_chain();
    VSIE_HIP(hipEventRecord(H.join, H.side));
  }
  volume_chain<R>(H, D, mn ? xn : nullptr, xb, yn, yb, st, T);
  if (conc)
    VSIE_HIP(hipStreamWaitEvent(st, H.join, 0));
  else if (mf)
    far_chain();
  // precorrection
  T.begin(9);
  launch_csr_add<R>(st, H.d_pc_rowid, H.d_pc_rowptr, H.d_pc_col, D.pc_val, x, y, H.n_pcrows);
  T.end(9);
  // ACA: y_n += U (V^* x_f), y_f += conj(V) (U^T x_n); V is read once for both
  if (mf && mn && H.aca_k > 0) {
    T.begin(10);
    cx<R>* part = D.small_work;
    cx<R>* tn = D.small_work + 512 * 256;
    cx<R>* tf = tn + 256;
    launch_lr_t<R>(st, false, D.U, xn, mn, H.aca_k, part, 512, tn);
    launch_lr_dual<R>(st, D.V, H.aca_k, mf, xf, tn, yf, D.dual_part, tf);
    launch_lr_n_add<R>(st, false, D.U, tf, mn, H.aca_k, yn);
    T.end(10);
  }
  // TT far coupling (eqs. (16)-(17)): the accumulation into y_b
  if (have_tt) {
    T.begin(13);
    launch_tt_post<R>(st, td, H.n, mf, H.d_mask, yb, D.tt_work);
    T.end(13);
  }
  T.collect();
}

// nrhs products: the dense far block, the largest operand, is read once per group of up to 16
// right-hand sides (each tile yields the partial sums of every column of the group); the rest
// of each product runs per column.
template <typename R> void matvec_batch(Handle& H, OpData<R>& D, const cx<R>* x, cx<R>* y, int nrhs, hipStream_t st) {
  constexpr int kGroup = 16;
  const int64_t N = H.N;
  const bool batched = nrhs > 1 && H.mf > 0;
  if (batched) {
    const int64_t nt = (int64_t)H.sym_T * (H.sym_T + 1) / 2;
    const int64_t ldp = nt * 2 * SYM_TB;
    if (!D.multi_part) D.multi_part = H.dalloc<cx<R>>(kGroup * ldp);
    for (int c0 = 0; c0 < nrhs; c0 += kGroup) {
      const int nb = std::min(kGroup, nrhs - c0);
      launch_symv_multi<R>(st, D.Zff, H.d_tiles, H.sym_T, x + c0 * N, N, H.mf, nb, D.multi_part, ldp);
      for (int b = 0; b < nb; ++b) launch_symv_reduce<R>(st, D.multi_part + b * ldp, H.sym_T, H.mf, y + (c0 + b) * N);
    }
  }
  for (int c = 0; c < nrhs; ++c) matvec_one<R>(H, D, x + c * N, y + c * N, st, batched);
}

// ---------------------------------------------------------------------------------------------
// Elimination of the far currents. The far conductor couples to the near currents and the body
// only through the ACA factors (eq. (12)) and the TT cores (eq. (14)), so its unknowns leave the
// system exactly through a K x K matrix, K = ACA rank + TT ranks r3 (the elimination the paper's
// conclusion proposes): Z_fr x_r = L t(x_r), L = [conj(V) | G4_0^T | G4_1^T | G4_2^T], and the
// reduced operator is Z_rr x_r - R^T S t(x_r) with S = L^T Z_ff^-1 L; R^T injects proxy values
// through the same factors in the forward direction.

// device buffer released at scope exit (setup temporaries)
struct Scratch {
  void* p = nullptr;
  explicit Scratch(size_t bytes) {
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
      p = nullptr;
      throw Error(VSIE_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  Scratch(Scratch&& o) noexcept : p(o.p) { o.p = nullptr; }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() {
    if (p) (void)hipFree(p);
  }
  template <typename T> T* as() const { return (T*)p; }
};

static int aca_rank(const Handle& H) { return (H.mf > 0 && H.mn > 0 && H.aca_k > 0) ? H.aca_k : 0; }
static OpData<double>& opdata(Handle& H, double) { return H.d64; }
static OpData<float>& opdata(Handle& H, float) { return H.d32; }
static Handle::SchurOp<double>& schurop(Handle& H, double) { return H.schur.d64; }
static Handle::SchurOp<float>& schurop(Handle& H, float) { return H.schur.d32; }

// C (M x N) = A B with explicit element strides (row, column) of each operand
static void gemm_strided(hipStream_t st, int M, int N, int K, const cxd* A, int64_t sar, int64_t sac, const cxd* B,
                         int64_t sbr, int64_t sbc, cxd* C, int64_t scr, int64_t scc, int accumulate, int negate) {
  GemmSet<double> G{};
  G.nprob = 1;
  G.nbatch[0] = 1;
  G.g[0] = GemmArgs<double>{A, sar, sac, 0, B, sbr, sbc, 0, C, scr, scc, 0, M, N, K, 0, nullptr, nullptr, accumulate,
                            negate};
  launch_zgemm<double>(st, G);
}

// y_n += U p_a and y_b += forward TT chain of p3 (eqs. (16)-(17) from the rank-r3 stage on)
template <typename R>
static void inject_proxies(Handle& H, const cx<R>* pa, const cx<R>* p3, cx<R>* yn, cx<R>* yb, hipStream_t st) {
  OpData<R>& D = opdata(H, R());
  TTDesc<R> td;
  int r3[3];
  const bool have_tt = tt_desc(H, D, td, r3);
  const int ka = aca_rank(H);
  if (ka) launch_lr_n_add<R>(st, false, D.U, pa, H.mn, ka, yn);
  if (have_tt) {
    launch_tt_forward_from<R>(st, td, H.n, H.mf, p3, D.tt_work);
    launch_tt_forward_post<R>(st, td, H.n, H.mf, H.d_mask, yb, D.tt_work);
  }
}

// ta = U^T x_n and s3 (start of the TT work buffer) = transpose TT chain of x_b: the proxies t(x_r)
template <typename R> static void far_proxies(Handle& H, const cx<R>* xn, const cx<R>* xb, hipStream_t st) {
  OpData<R>& D = opdata(H, R());
  TTDesc<R> td;
  int r3[3];
  const bool have_tt = tt_desc(H, D, td, r3);
  const int ka = aca_rank(H);
  if (ka) launch_lr_t<R>(st, false, D.U, xn, H.mn, ka, D.small_work, 512, schurop(H, R()).ta);
  if (have_tt) launch_tt_transpose_pre<R>(st, td, H.n, H.mf, xb, body_mask(H), D.tt_work);
}

// Reduced product y_r = Z_rr x_r - R^T S t(x_r) on the near and body unknowns (x_f is not read,
// y_f is set to zero), in FP64 or complex64.
template <typename R> static void matvec_schur(Handle& H, const cx<R>* x, cx<R>* y, hipStream_t st) {
  OpData<R>& D = opdata(H, R());
  Handle::SchurOp<R>& P = schurop(H, R());
  const int K = H.schur.K;
  StageTimer T(H, st);
  const int mf = H.mf, mn = H.mn;
  const cx<R>* xn = x + mf;
  const cx<R>* xb = x + mf + mn;
  cx<R>* yn = y + mf;
  cx<R>* yb = y + mf + mn;
  // the proxy chain reads only x and writes only its own buffers, so it runs on the second stream
  // beside the volume chain; the injections into y_n and y_b follow the join
  TTDesc<R> td;
  int r3[3];
  const bool have_tt = tt_desc(H, D, td, r3);
  const int ka = aca_rank(H);
  if (K > 0) {
    if (!H.side) make_streams(H);
    VSIE_HIP(hipEventRecord(H.fork, st));
    VSIE_HIP(hipStreamWaitEvent(H.side, H.fork, 0));
    T.begin(10, H.side);
    far_proxies<R>(H, xn, xb, H.side);
    launch_schur_apply<R>(H.side, P.S, K, ka, r3, P.ta, D.tt_work, (R)-1, P.pa, P.p3);
    if (have_tt) launch_tt_forward_from<R>(H.side, td, H.n, H.mf, P.p3, D.tt_work);
    T.end(10, H.side);
    VSIE_HIP(hipEventRecord(H.join, H.side));
  }
  volume_chain<R>(H, D, mn ? xn : nullptr, xb, yn, yb, st, T);
  T.begin(9);
  launch_csr_add<R>(st, H.d_pc_rowid, H.d_pc_rowptr, H.d_pc_col, D.pc_val, x, y, H.n_pcrows);
  T.end(9);
  if (K > 0) {
    VSIE_HIP(hipStreamWaitEvent(st, H.join, 0));
    T.begin(13);
    if (ka) launch_lr_n_add<R>(st, false, D.U, P.pa, H.mn, ka, yn);
    if (have_tt) launch_tt_forward_post<R>(st, td, H.n, H.mf, H.d_mask, yb, D.tt_work);
    T.end(13);
  }
  if (mf) VSIE_HIP(hipMemsetAsync(y, 0, sizeof(cx<R>) * mf, st));
  T.collect();
}

// Right preconditioner of the reduced system: the inverse of its near block (direct Galerkin
// entries of the near coils minus the eliminated far block's ACA term) on the near currents, the
// inverse diagonal on the body unknowns, zero on the far currents. Identity (zero on the far
// currents) when `use` is false or the preconditioner is not built.
template <typename R>
static void precond_apply(Handle& H, const cx<R>* v, cx<R>* w, hipStream_t st, bool use = true) {
  Handle::Schur& Sc = H.schur;
  Handle::SchurOp<R>& P = schurop(H, R());
  const int mf = H.mf, mn = H.mn;
  if (!use || !Sc.precond) {
    VSIE_HIP(hipMemcpyAsync(w, v, sizeof(cx<R>) * H.N, hipMemcpyDeviceToDevice, st));
    if (mf) VSIE_HIP(hipMemsetAsync(w, 0, sizeof(cx<R>) * mf, st));
    return;
  }
  if (mf) VSIE_HIP(hipMemsetAsync(w, 0, sizeof(cx<R>) * mf, st));
  if (mn) {
    launch_symv_tiles<R>(st, P.Xn, Sc.d_tiles_n, Sc.Tn, v + mf, mn, P.part_n);
    launch_symv_reduce<R>(st, P.part_n, Sc.Tn, mn, w + mf);
  }
  launch_mul_diag<R>(st, v + mf + mn, P.invdiag, w + mf + mn, 3LL * H.nv);
}

static std::vector<int> upper_tiles(int T) {
  std::vector<int> tiles;
  for (int I = 0; I < T; ++I)
    for (int J = I; J < T; ++J) {
      tiles.push_back(I);
      tiles.push_back(J);
    }
  return tiles;
}

static void setup_schur(Handle& H, bool precond) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = H.stream;
  OpData<double>& D = H.d64;
  Handle::Schur& Sc = H.schur;
  const int mf = H.mf, mn = H.mn;
  TTDesc<double> td;
  int r3[3];
  tt_desc(H, D, td, r3);
  const int ka = aca_rank(H);
  if (!Sc.ready) {
    Sc.K = mf ? ka + r3[0] + r3[1] + r3[2] : 0;
    if (Sc.K > 256 + 3 * TT_RMAX) throw Error(VSIE_E_ARG, "too many far-coupling proxies");
    Sc.d64.ta = H.dalloc<cxd>(256);
    Sc.d64.pa = H.dalloc<cxd>(256);
    Sc.d64.p3 = H.dalloc<cxd>(3 * TT_RMAX);
    Sc.tc = H.dalloc<cxd>(std::max(Sc.K, 1));
    for (auto& v : Sc.vec) v = H.dalloc<cxd>(H.N);
    if (mf) {
      // dense far block from its tiles, factored in place
      Sc.zf = H.dalloc<cxd>(mf);
      DenseLU& F = Sc.ff;
      F.n = mf;
      F.lda = mf;
      F.A = H.dalloc<cxd>((int64_t)mf * mf);
      F.Linv = H.dalloc<cxd>(lu_blocks_elems(mf));
      F.Uinv = H.dalloc<cxd>(lu_blocks_elems(mf));
      F.d_ipiv = H.dalloc<int>(mf);
      F.d_perm = H.dalloc<int>(mf);
      F.d_info = H.dalloc<int>(1);
      launch_unpack_sym(st, D.Zff, H.sym_T, mf, F.A);
      {
        Scratch work(sizeof(cxd) * lu_work_elems(mf));
        lu_factor(st, F, work.as<cxd>());
      }
      if (Sc.K > 0) {
        const int K = Sc.K;
        Scratch L(sizeof(cxd) * mf * K), Wt(sizeof(cxd) * mf * K);
        launch_build_far_factors(st, D.V, ka, td, mf, K, L.as<cxd>());
        Sc.W = H.dalloc<cxd>((int64_t)mf * K);
        VSIE_HIP(hipMemcpyAsync(Sc.W, L.p, sizeof(cxd) * mf * K, hipMemcpyDeviceToDevice, st));
        lu_solve(st, F, Sc.W, K, K, Wt.as<cxd>());
        // S = L^T W
        Sc.d64.S = H.dalloc<cxd>((int64_t)K * K);
        gemm_strided(st, K, K, mf, L.as<cxd>(), 1, K, Sc.W, K, 1, Sc.d64.S, K, 1, 0, 0);
        VSIE_HIP(hipGetLastError());
        VSIE_HIP(hipStreamSynchronize(st));
      }
    }
    Sc.ready = true;
  }
  if (precond && !Sc.precond) {
    if (mn) {
      // reduced near block: direct Galerkin entries minus U S_aa U^T, inverted through its LU
      Scratch Zn(sizeof(cxd) * mn * mn), X(sizeof(cxd) * mn * mn);
      launch_zcc_dense(st, H.dnear, H.dnear, H.k0, 0, mn, Zn.as<cxd>());
      if (ka && Sc.K > 0) {
        Scratch T1(sizeof(cxd) * mn * ka);
        gemm_strided(st, mn, ka, ka, D.U, 1, mn, Sc.d64.S, Sc.K, 1, T1.as<cxd>(), ka, 1, 0, 0);
        gemm_strided(st, mn, mn, ka, T1.as<cxd>(), ka, 1, D.U, mn, 1, Zn.as<cxd>(), mn, 1, 1, 1);
        VSIE_HIP(hipStreamSynchronize(st));
      }
      DenseLU F;
      F.n = mn;
      F.lda = mn;
      F.A = Zn.as<cxd>();
      Scratch Li(sizeof(cxd) * lu_blocks_elems(mn)), Ui(sizeof(cxd) * lu_blocks_elems(mn)),
          ip(sizeof(int) * mn), pm(sizeof(int) * mn), inf(sizeof(int)), work(sizeof(cxd) * lu_work_elems(mn));
      F.Linv = Li.as<cxd>();
      F.Uinv = Ui.as<cxd>();
      F.d_ipiv = ip.as<int>();
      F.d_perm = pm.as<int>();
      F.d_info = inf.as<int>();
      lu_factor(st, F, work.as<cxd>());
      launch_set_identity(st, X.as<cxd>(), mn);
      {
        Scratch Wn(sizeof(cxd) * mn * mn);
        lu_solve(st, F, X.as<cxd>(), mn, mn, Wn.as<cxd>());
        VSIE_HIP(hipStreamSynchronize(st));
      }
      Sc.Tn = (mn + SYM_TB - 1) / SYM_TB;
      const std::vector<int> tiles = upper_tiles(Sc.Tn);
      const int64_t nt = (int64_t)tiles.size() / 2;
      Sc.d_tiles_n = upload(H, tiles);
      Sc.d64.Xn = H.dalloc<cxd>(nt * SYM_TB * SYM_TB);
      Sc.d64.part_n = H.dalloc<cxd>(nt * 2 * SYM_TB);
      launch_pack_sym(st, X.as<cxd>(), mn, Sc.d_tiles_n, nt, Sc.d64.Xn);
      VSIE_HIP(hipGetLastError());
      VSIE_HIP(hipStreamSynchronize(st));
    }
    // body diagonal: h^3 / chi + h^3 T_aa(0) (the self term of the convolution), 1 in air
    cxd T0[3];
    for (int a = 0; a < 3; ++a)
      VSIE_HIP(hipMemcpy(&T0[a], H.d_oct + (int64_t)a * H.Ne, sizeof(cxd), hipMemcpyDeviceToHost));
    const double h3 = H.h * H.h * H.h;
    std::vector<cxd> inv(3 * (size_t)H.nv, cxd{1, 0});
    for (int p = 0; p < H.nv; ++p)
      if (H.chi[p].re != 0 || H.chi[p].im != 0)
        for (int a = 0; a < 3; ++a) inv[(size_t)a * H.nv + p] = cinv(h3 * cinv(H.chi[p]) + h3 * T0[a]);
    Sc.d64.invdiag = upload_cx<double>(H, inv);
    build_material(H, inv);
    Sc.precond = true;
  }
  // complex64 copies for the mixed-precision solve
  if (H.have32 && !Sc.d32.ta) {
    Sc.d32.ta = H.dalloc<cxf>(256);
    Sc.d32.pa = H.dalloc<cxf>(256);
    Sc.d32.p3 = H.dalloc<cxf>(3 * TT_RMAX);
    if (Sc.K > 0) {
      Sc.d32.S = H.dalloc<cxf>((int64_t)Sc.K * Sc.K);
      launch_d2f(st, Sc.d64.S, Sc.d32.S, (int64_t)Sc.K * Sc.K);
    }
  }
  if (H.have32 && Sc.precond && !Sc.d32.invdiag) {
    if (mn) {
      const int64_t nt = (int64_t)Sc.Tn * (Sc.Tn + 1) / 2;
      Sc.d32.Xn = H.dalloc<cxf>(nt * SYM_TB * SYM_TB);
      Sc.d32.part_n = H.dalloc<cxf>(nt * 2 * SYM_TB);
      launch_d2f(st, Sc.d64.Xn, Sc.d32.Xn, nt * SYM_TB * SYM_TB);
    }
    Sc.d32.invdiag = H.dalloc<cxf>(3LL * H.nv);
    launch_d2f(st, Sc.d64.invdiag, Sc.d32.invdiag, 3LL * H.nv);
    VSIE_HIP(hipStreamSynchronize(st));
  }
  Sc.seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------------------------
// GMRES (FP64 Arnoldi, classical Gram-Schmidt with selective reorthogonalisation) with a matvec
// callback on FP64 vectors
static bool verbose() {
  static const bool on = getenv("VSIE_VERBOSE") != nullptr;
  return on;
}

constexpr int IR_OUTER_M = 20;   // FP64 flexible-GMRES steps per cycle of the mixed-precision solver

struct Solver {
  Handle& H;
  hipStream_t st;
  int64_t N;
  cxd* part;     // multidot partials [MDOT_BLK][MAX_BASIS + 3]
  cxd* sum;      // their sums (h, then the segment norms)
  cxd* npart2;   // norm partials of the update [NB2][3]
  cxd* nsum;
  double* npart;
  static constexpr int NBLK = 256;
  static constexpr int MDOT_BLK = 1024;
  static constexpr int NB2 = 1024;
  static constexpr int MAX_BASIS = 1024;
  // layout of the page-locked buffer: projection sums [0, MAX_BASIS + 3), update norms, segment norms
  static constexpr int PIN_NSUM = MAX_BASIS + 3;
  static constexpr int PIN_NORMS = PIN_NSUM + 3;
  static_assert(PIN_NORMS + (3 * NBLK + 1) / 2 <= Handle::HOST_PINNED_ELEMS, "page-locked buffer too small");
  static int64_t work_elems() { return (int64_t)MDOT_BLK * (MAX_BASIS + 3) + (MAX_BASIS + 3) + 3 * NB2 + 3; }
  double kappa = 0.1;          // second Gram-Schmidt pass when a pass leaves less than kappa ||w||
  int64_t second_passes = 0;   // Arnoldi steps that took it
  Solver(Handle& h, hipStream_t s) : H(h), st(s), N(h.n_active) {
    part = H.d_solve_work;
    sum = part + (int64_t)MDOT_BLK * (MAX_BASIS + 3);
    npart2 = sum + MAX_BASIS + 3;
    nsum = npart2 + 3 * NB2;
    npart = H.d_red;
  }
  // segment norms (far, near, body) and the total of a compact (n < 0) or full-length vector
  void norms(const cxd* a, double out[4], int64_t n = -1) {
    launch_norm_partial(st, a, n < 0 ? N : n, H.mf, (int64_t)H.mf + H.mn, npart, NBLK);
    const double* p = reinterpret_cast<const double*>(H.h_pinned + PIN_NORMS);
    VSIE_HIP(hipMemcpyAsync(H.h_pinned + PIN_NORMS, npart, sizeof(double) * 3 * NBLK, hipMemcpyDeviceToHost, st));
    VSIE_HIP(hipStreamSynchronize(st));
    double s[3] = {0, 0, 0};
    for (int b = 0; b < NBLK; ++b)
      for (int q = 0; q < 3; ++q) s[q] += p[3 * b + q];
    out[0] = sqrt(s[0]);
    out[1] = sqrt(s[1]);
    out[2] = sqrt(s[2]);
    out[3] = sqrt(s[0] + s[1] + s[2]);
  }
  // Classical Gram-Schmidt of w against V[0..nvec): one pass forms h = V^H w (with the segment
  // norms of w on the first pass), a second applies w -= V h with the device copy of h and forms
  // the norms of the result; repeated once when the first pass left less than kappa of the norm
  // of w (the DGKS test; its classical constant is 1/sqrt(2), the default here 0.1: a single pass
  // that keeps a tenth of the norm loses at most about ten roundings of orthogonality). One host
  // synchronisation per pass. h receives the projection coefficients; the return value is ||w||
  // afterwards.
  double orthogonalize(const cxd* V, int nvec, cxd* w, std::vector<cxd>& h) {
    if (nvec > MAX_BASIS) throw Error(VSIE_E_ARG, "Krylov basis larger than 1024 vectors");
    const int64_t s1 = H.mf, s2 = (int64_t)H.mf + H.mn;
    h.assign(nvec, cxd{0, 0});
    double n0 = 0, n1 = 0;
    // the reductions come back through page-locked memory: truly asynchronous copies, one wait
    const cxd* hh = H.h_pinned;
    const cxd* nn = H.h_pinned + PIN_NSUM;
    for (int pass = 0; pass < 2; ++pass) {
      const int K = nvec + (pass == 0 ? 3 : 0);
      launch_multidot(st, V, N, nvec, w, N, s1, s2, pass == 0, part, MDOT_BLK);
      launch_sum_partials(st, part, MDOT_BLK, K, sum);
      launch_multiaxpy_norm(st, V, N, nvec, sum, w, N, s1, s2, npart2, NB2);
      launch_sum_partials(st, npart2, NB2, 3, nsum);
      VSIE_HIP(hipMemcpyAsync(H.h_pinned, sum, sizeof(cxd) * K, hipMemcpyDeviceToHost, st));
      VSIE_HIP(hipMemcpyAsync(H.h_pinned + PIN_NSUM, nsum, sizeof(cxd) * 3, hipMemcpyDeviceToHost, st));
      VSIE_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < nvec; ++i) h[i] += hh[i];
      if (pass == 0) n0 = sqrt(hh[nvec].re + hh[nvec + 1].re + hh[nvec + 2].re);
      n1 = sqrt(nn[0].re + nn[1].re + nn[2].re);
      if (n1 >= kappa * n0) break;
      if (pass == 0) ++second_passes;
    }
    return n1;
  }
  // solve A x = b to relative residual tol (x initialised to zero). Returns iterations used.
  template <typename MV>
  int gmres(MV&& A, const cxd* b, cxd* x, double tol, int restart, int max_iter, int* restarts, double* relres,
            cxd* Vbuf, cxd* w, cxd* hvec_dev) {
    VSIE_HIP(hipMemsetAsync(x, 0, sizeof(cxd) * N, st));
    double nb[4];
    norms(b, nb);
    const double bnorm = nb[3];
    *relres = 0;
    if (bnorm == 0) return 0;
    int it = 0;
    std::vector<cxd> Hm((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h;
    for (;;) {
      A(x, w);
      launch_sub(st, b, w, w, N);      // r = b - A x
      double nr[4];
      norms(w, nr);
      *relres = nr[3] / bnorm;
      if (verbose()) {
        fprintf(stderr, "[vsie] gmres: %d iterations, true relative residual %.3e\n", it, *relres);
        fflush(stderr);
      }
      if (*relres <= tol || it >= max_iter) break;
      ++*restarts;
      const double beta = nr[3];
      launch_scale_copy(st, w, 1.0 / beta, Vbuf, N);
      std::fill(g.begin(), g.end(), cxd{0, 0});
      g[0] = {beta, 0};
      int jend = 0;
      bool done = false;
      for (int j = 0; j < restart; ++j) {
        A(Vbuf + (int64_t)j * N, w);
        double nw[4] = {0, 0, 0, orthogonalize(Vbuf, j + 1, w, h)};
        for (int i = 0; i <= j; ++i) Hm[(size_t)i * restart + j] = h[i];
        Hm[(size_t)(j + 1) * restart + j] = {nw[3], 0};
        if (nw[3] > 0) launch_scale_copy(st, w, 1.0 / nw[3], Vbuf + (int64_t)(j + 1) * N, N);
        for (int i = 0; i < j; ++i) {
          cxd a = Hm[(size_t)i * restart + j], bb = Hm[(size_t)(i + 1) * restart + j];
          Hm[(size_t)i * restart + j] = conj(cs[i]) * a + conj(sn[i]) * bb;
          Hm[(size_t)(i + 1) * restart + j] = cxd{-sn[i].re, -sn[i].im} * a + cs[i] * bb;
        }
        cxd a = Hm[(size_t)j * restart + j], bb = Hm[(size_t)(j + 1) * restart + j];
        double den = sqrt(a.re * a.re + a.im * a.im + bb.re * bb.re + bb.im * bb.im);
        cs[j] = den > 0 ? (1.0 / den) * a : cxd{1, 0};
        sn[j] = den > 0 ? (1.0 / den) * bb : cxd{0, 0};
        Hm[(size_t)j * restart + j] = conj(cs[j]) * a + conj(sn[j]) * bb;
        Hm[(size_t)(j + 1) * restart + j] = {0, 0};
        g[j + 1] = cxd{-sn[j].re, -sn[j].im} * g[j];
        g[j] = conj(cs[j]) * g[j];
        ++it;
        jend = j + 1;
        double est = sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im) / bnorm;
        if (est <= tol || it >= max_iter || nw[3] == 0) {
          done = true;
          break;
        }
      }
      // back substitution
      std::vector<cxd> y(jend);
      for (int i = jend - 1; i >= 0; --i) {
        cxd s = g[i];
        for (int k = i + 1; k < jend; ++k) s -= Hm[(size_t)i * restart + k] * y[k];
        y[i] = s * cinv(Hm[(size_t)i * restart + i]);
      }
      VSIE_HIP(hipMemcpyAsync(hvec_dev, y.data(), sizeof(cxd) * jend, hipMemcpyHostToDevice, st));
      launch_combine_add(st, Vbuf, N, jend, hvec_dev, x, N);
      (void)done;
    }
    return it;
  }

  // Flexible GMRES in FP64 whose preconditioner P(v, z) may change from step to step (here an
  // inner complex64 GMRES solve of Z z = v). Vb holds m + 1 basis vectors, Zb the m
  // preconditioned ones; x = sum_j Zb_j y_j minimises the FP64 residual over their span. With an
  // exact inner solve one step is one refinement x += Z^{-1} r. P returns false when the inner
  // iteration budget is spent.
  template <class MV, class PC>
  int fgmres(MV&& A, PC&& P, const cxd* b, cxd* x, double tol, int m, int* steps, double* relres, cxd* Vb, cxd* Zb,
             cxd* w, cxd* hvec_dev) {
    VSIE_HIP(hipMemsetAsync(x, 0, sizeof(cxd) * N, st));
    double nb[4];
    norms(b, nb);
    const double bnorm = nb[3];
    *relres = 0;
    if (bnorm == 0) return 0;
    std::vector<cxd> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h;
    bool budget = true;
    int cycles = 0;
    for (;;) {
      A(x, w);
      launch_sub(st, b, w, w, N);
      double nr[4];
      norms(w, nr);
      *relres = nr[3] / bnorm;
      if (verbose()) {
        fprintf(stderr, "[vsie] flexible GMRES: %d FP64 steps, true relative residual %.3e\n", *steps, *relres);
        fflush(stderr);
      }
      if (*relres <= tol || !budget || cycles >= 100) break;
      ++cycles;
      const double beta = nr[3];
      launch_scale_copy(st, w, 1.0 / beta, Vb, N);
      std::fill(g.begin(), g.end(), cxd{0, 0});
      g[0] = {beta, 0};
      int jend = 0;
      for (int j = 0; j < m; ++j) {
        cxd* z = Zb + (int64_t)j * N;
        budget = P(Vb + (int64_t)j * N, z);
        A(z, w);
        double nw[4] = {0, 0, 0, orthogonalize(Vb, j + 1, w, h)};
        for (int i = 0; i <= j; ++i) Hm[(size_t)i * m + j] = h[i];
        Hm[(size_t)(j + 1) * m + j] = {nw[3], 0};
        if (nw[3] > 0) launch_scale_copy(st, w, 1.0 / nw[3], Vb + (int64_t)(j + 1) * N, N);
        for (int i = 0; i < j; ++i) {
          cxd a = Hm[(size_t)i * m + j], bb = Hm[(size_t)(i + 1) * m + j];
          Hm[(size_t)i * m + j] = conj(cs[i]) * a + conj(sn[i]) * bb;
          Hm[(size_t)(i + 1) * m + j] = cxd{-sn[i].re, -sn[i].im} * a + cs[i] * bb;
        }
        cxd a = Hm[(size_t)j * m + j], bb = Hm[(size_t)(j + 1) * m + j];
        double den = sqrt(a.re * a.re + a.im * a.im + bb.re * bb.re + bb.im * bb.im);
        cs[j] = den > 0 ? (1.0 / den) * a : cxd{1, 0};
        sn[j] = den > 0 ? (1.0 / den) * bb : cxd{0, 0};
        Hm[(size_t)j * m + j] = conj(cs[j]) * a + conj(sn[j]) * bb;
        Hm[(size_t)(j + 1) * m + j] = {0, 0};
        g[j + 1] = cxd{-sn[j].re, -sn[j].im} * g[j];
        g[j] = conj(cs[j]) * g[j];
        ++*steps;
        jend = j + 1;
        double est = sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im) / bnorm;
        if (est <= tol || !budget || nw[3] == 0) break;
      }
      std::vector<cxd> y(jend);
      for (int i = jend - 1; i >= 0; --i) {
        cxd sacc = g[i];
        for (int k = i + 1; k < jend; ++k) sacc -= Hm[(size_t)i * m + k] * y[k];
        y[i] = sacc * cinv(Hm[(size_t)i * m + i]);
      }
      VSIE_HIP(hipMemcpyAsync(hvec_dev, y.data(), sizeof(cxd) * jend, hipMemcpyHostToDevice, st));
      launch_combine_add(st, Zb, N, jend, hvec_dev, x, N);
    }
    return *steps;
  }
};

void ensure_solver_ws(Handle& H, int restart) {
  if (!H.d_solve_work) {
    H.d_solve_work = H.dalloc<cxd>(Solver::work_elems());
    H.d_red = H.dalloc<double>(256 * 4);
  }
  if (!H.h_pinned && hipHostMalloc((void**)&H.h_pinned, sizeof(cxd) * Handle::HOST_PINNED_ELEMS, hipHostMallocDefault) != hipSuccess) {
    H.h_pinned = nullptr;
    throw Error(VSIE_E_NOMEM, "page-locked host buffer of the solver");
  }
  if (!H.d_active) {
    std::vector<int> act;
    act.reserve((size_t)H.mf + H.mn + 3 * H.tissue.size());
    for (int i = 0; i < H.mf + H.mn; ++i) act.push_back(i);
    for (int c = 0; c < 3; ++c)
      for (int p = 0; p < H.nv; ++p)
        if (H.chi[p].re != 0 || H.chi[p].im != 0) act.push_back((int)(H.mf + H.mn + (int64_t)c * H.nv + p));
    H.n_active = (int64_t)act.size();
    H.d_active = upload(H, act);
    for (auto& v : H.d_full) v = H.dalloc<cxd>(H.N);
    VSIE_HIP(hipMemset(H.d_full[0], 0, sizeof(cxd) * H.N));
  }
  if (H.krylov_cols < restart + 1) {
    if (H.d_krylov) {
      auto it = std::find(H.allocations.begin(), H.allocations.end(), (void*)H.d_krylov);
      if (it != H.allocations.end()) H.allocations.erase(it);
      H.device_bytes -= (int64_t)sizeof(cxd) * H.krylov_cols * H.n_active;
      VSIE_HIP(hipFree(H.d_krylov));
      H.d_krylov = nullptr;
    }
    H.d_krylov = H.dalloc<cxd>((int64_t)(restart + 1) * H.n_active);
    H.krylov_cols = restart + 1;
  }
}

// Work buffers of the solvers: compact vectors (coupled unknowns) and, for the mixed-precision
// methods, the flexible-GMRES bases and full-length complex64 product vectors.
struct SolveWork {
  cxd *wc, *bc, *xc, *dc, *hv, *hv2, *Vout, *Zout;
  cxf *x32, *y32;
};

// GMRES on the reduced system (far currents eliminated), right-preconditioned when the
// preconditioner is built: solve (A_S M) u = b_r - Z_rf Z_ff^-1 b_f on the compact unknowns,
// x_r = M u, then recover x_f = Z_ff^-1 (b_f - L t(x_r)); air voxels take x = b.
// mixed: FP64 flexible GMRES whose preconditioner is one complex64 GMRES cycle on the complex64
// reduced operator (at most `restart` iterations, stopping at inner_tol). Returns the iterations
// (inner ones when mixed); *outer receives the FP64 flexible steps.
int solve_schur(Handle& H, Solver& S, const vsie_solve_opts& so, bool mixed, const cxd* b, cxd* x,
                const SolveWork& ws, int* restarts, int* outer, double* rel, hipStream_t st) {
  Handle::Schur& Sc = H.schur;
  OpData<double>& D = H.d64;
  const int64_t N = H.N, Nc = H.n_active;
  const int mf = H.mf, mn = H.mn, K = Sc.K, ka = aca_rank(H);
  const bool use_pc = so.precond != 0;
  TTDesc<double> td;
  int r3[3];
  tt_desc(H, D, td, r3);
  cxd* bred = Sc.vec[0];
  cxd* tmp = Sc.vec[1];
  cxd* fin = H.d_full[0];
  cxd* fout = H.d_full[1];
  double nb[4], nbr[4];
  S.norms(b, nb, N);
  const bool bf = mf > 0 && nb[0] > 0;
  VSIE_HIP(hipMemcpyAsync(bred, b, sizeof(cxd) * N, hipMemcpyDeviceToDevice, st));
  if (mf) VSIE_HIP(hipMemsetAsync(bred, 0, sizeof(cxd) * mf, st));
  if (bf) {
    VSIE_HIP(hipMemcpyAsync(Sc.zf, b, sizeof(cxd) * mf, hipMemcpyDeviceToDevice, st));
    lu_solve(st, Sc.ff, Sc.zf, 1, 1, tmp);
    if (K) {
      // proxies of Z_ff^-1 b_f: L^T Z_ff^-1 b_f = W^T b_f, injected with a minus sign
      gemm_strided(st, K, 1, mf, Sc.W, 1, K, b, 1, 1, Sc.tc, 1, 1, 0, 0);
      launch_schur_scatter(st, K, ka, r3, Sc.tc, -1.0, Sc.d64.pa, Sc.d64.p3);
      inject_proxies<double>(H, Sc.d64.pa, Sc.d64.p3, bred + mf, bred + mf + mn, st);
    }
  }
  launch_gather_idx(st, bred, H.d_active, Nc, ws.bc);
  S.norms(ws.bc, nbr);
  const double tol = nbr[3] > 0 ? so.tol * nb[3] / nbr[3] : so.tol;
  auto AM = [&](const cxd* in, cxd* out) {
    launch_scatter_idx(st, in, H.d_active, Nc, fin);
    precond_apply<double>(H, fin, tmp, st, use_pc);
    matvec_schur<double>(H, tmp, fout, st);
    // training pairs of the learned preconditioner: z = M v with its exact image A_S z
    if (H.collect && use_pc && Sc.precond) net_collect_pair(H, *H.collect, tmp, fout, Sc.vec[2], st);
    launch_gather_idx(st, fout, H.d_active, Nc, out);
  };
  int it = 0;
  const bool learned = so.method == VSIE_SCHUR_LEARNED;
  if (learned) {
    // flexible GMRES on A_S x = b_r with the preconditioner P(v) = M v + learned body correction
    auto AS = [&](const cxd* in, cxd* out) {
      launch_scatter_idx(st, in, H.d_active, Nc, fin);
      matvec_schur<double>(H, fin, fout, st);
      launch_gather_idx(st, fout, H.d_active, Nc, out);
    };
    auto PL = [&](const cxd* v, cxd* z) {
      launch_scatter_idx(st, v, H.d_active, Nc, fin);
      precond_apply<double>(H, fin, tmp, st, true);
      net_apply(H, *H.net, fin, tmp, st);
      launch_gather_idx(st, tmp, H.d_active, Nc, z);
      ++it;
      return it < so.max_iter;
    };
    int steps = 0;
    S.fgmres(AS, PL, ws.bc, ws.xc, tol, so.restart, &steps, rel, ws.Vout, ws.Zout, ws.wc, ws.hv);
    *outer = steps;
  } else if (!mixed) {
    it = S.gmres(AM, ws.bc, ws.xc, tol, so.restart, so.max_iter, restarts, rel, H.d_krylov, ws.wc, ws.hv);
  } else {
    // complex64 product of the preconditioned reduced operator on compact FP64 vectors
    auto AM32 = [&](const cxd* in, cxd* out) {
      launch_scatter_idx(st, in, H.d_active, Nc, fin);
      launch_d2f(st, fin, ws.x32, N);
      precond_apply<float>(H, ws.x32, ws.y32, st, use_pc);
      matvec_schur<float>(H, ws.y32, ws.x32, st);
      launch_f2d(st, ws.x32, fout, N);
      launch_gather_idx(st, fout, H.d_active, Nc, out);
    };
    auto P32 = [&](const cxd* v, cxd* z) {
      double inner_rel = 0;
      const int used = S.gmres(AM32, v, z, so.inner_tol, so.restart,
                               std::max(1, std::min(so.restart, so.max_iter - it)), restarts, &inner_rel, H.d_krylov,
                               ws.dc, ws.hv2);
      it += used;
      return it < so.max_iter;
    };
    S.fgmres(AM, P32, ws.bc, ws.xc, tol, IR_OUTER_M, outer, rel, ws.Vout, ws.Zout, ws.wc, ws.hv);
  }
  // x = M u on the coupled unknowns (the flexible method's iterate is x itself), b on the air voxels
  if (learned) {
    VSIE_HIP(hipMemcpyAsync(ws.wc, ws.xc, sizeof(cxd) * Nc, hipMemcpyDeviceToDevice, st));
  } else {
    launch_scatter_idx(st, ws.xc, H.d_active, Nc, fin);
    precond_apply<double>(H, fin, tmp, st, use_pc);
    launch_gather_idx(st, tmp, H.d_active, Nc, ws.wc);
  }
  VSIE_HIP(hipMemcpyAsync(x, b, sizeof(cxd) * N, hipMemcpyDeviceToDevice, st));
  launch_scatter_idx(st, ws.wc, H.d_active, Nc, x);
  if (mf) {
    if (bf) VSIE_HIP(hipMemcpyAsync(x, Sc.zf, sizeof(cxd) * mf, hipMemcpyDeviceToDevice, st));
    if (K) {
      far_proxies<double>(H, x + mf, x + mf + mn, st);
      launch_schur_gather(st, K, ka, r3, Sc.d64.ta, D.tt_work, -1.0, Sc.tc);
      launch_gemv_rows<double>(st, Sc.W, Sc.tc, mf, K, x, 1);
    }
  }
  VSIE_HIP(hipGetLastError());
  return it;
}

__global__ void k_zero_words(uint64_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// delta-gap right-hand side of one port from the device tables: zero fill, then the port's edges
void port_rhs(const Handle& H, int port, int dtype, void* b, hipStream_t st) {
  const int64_t words = (dtype == VSIE_C128 ? 2 : 1) * H.N;   // 8-byte words of N complex values
  const unsigned blocks = (unsigned)std::min<int64_t>((words + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, (uint64_t*)b, words);
  const int e0 = H.port_off[port], ne = H.port_off[port + 1] - e0;
  if (dtype == VSIE_C128)
    launch_scatter_rhs<double>(st, H.d_port_idx + e0, H.d_port_re + e0, H.d_port_im + e0, ne, (cxd*)b);
  else
    launch_scatter_rhs<float>(st, H.d_port_idx + e0, H.d_port_re + e0, H.d_port_im + e0, ne, (cxf*)b);
}

}  // namespace

// =============================================================================================
extern "C" {

int vsie_default_options(vsie_options* o) {
  if (!o) return fail(VSIE_E_ARG, "null options");
  o->tt_tol = 1e-3;
  o->tt_rank_max = 96;
  o->aca_tol = 1e-3;
  o->aca_rank_max = 256;
  o->precorrect_dist = 2;
  o->precision = VSIE_PREC_MIXED;
  o->build_far = 1;
  o->seed = 1;
  o->basis = VSIE_BASIS_PWC;
  o->stencil = 5;
  o->quad_near_vol = 8;
  o->quad_near_surf = 5;
  o->quad_far_vol = 1;
  o->quad_far_surf = 1;
  return VSIE_OK;
}

int vsie_default_solve_opts(vsie_solve_opts* o) {
  if (!o) return fail(VSIE_E_ARG, "null options");
  o->tol = 1e-6;
  o->restart = 50;
  o->max_iter = 5000;
  o->method = VSIE_GMRES64;
  o->inner_tol = 1e-3;
  o->precond = 1;
  o->reorth = 0.1;
  return VSIE_OK;
}

static void progress(const char* what, std::chrono::steady_clock::time_point t0) {
  if (!verbose()) return;
  double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fprintf(stderr, "[vsie] %7.2f s  %s\n", s, what);
  fflush(stderr);
}

static int create_impl(const vsie_problem* p, const vsie_options* opts, void* stream, vsie_handle* donor,
                       vsie_handle** out);

// 64-bit FNV-1a over the inputs that fix the TT and ACA factors: grid, materials, meshes (with
// their ports), frequency, and the compression options (tolerances, rank caps, seed)
static uint64_t input_hash(const vsie_problem* p, const vsie_options& o) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* data, size_t n) {
    const unsigned char* c = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  mix(p->n, sizeof(p->n));
  mix(&p->h, sizeof(double));
  mix(p->origin, sizeof(p->origin));
  mix(&p->freq_hz, sizeof(double));
  const size_t nv = (size_t)p->n[0] * p->n[1] * p->n[2];
  if (p->eps_r) mix(p->eps_r, sizeof(double) * nv);
  if (p->sigma) mix(p->sigma, sizeof(double) * nv);
  mix(&p->n_meshes, sizeof(int32_t));
  for (int i = 0; i < p->n_meshes && p->meshes; ++i) {
    const vsie_mesh& m = p->meshes[i];
    mix(&m.n_verts, sizeof(int32_t));
    mix(&m.n_tris, sizeof(int32_t));
    mix(&m.domain, sizeof(int32_t));
    mix(&m.n_port_edges, sizeof(int32_t));
    if (m.verts && m.n_verts > 0) mix(m.verts, sizeof(double) * 3 * (size_t)m.n_verts);
    if (m.tris && m.n_tris > 0) mix(m.tris, sizeof(int32_t) * 3 * (size_t)m.n_tris);
    if (m.port_edges && m.n_port_edges > 0) mix(m.port_edges, sizeof(int32_t) * 2 * (size_t)m.n_port_edges);
    if (m.port_id && m.n_port_edges > 0) mix(m.port_id, sizeof(int32_t) * (size_t)m.n_port_edges);
  }
  mix(&o.tt_tol, sizeof(double));
  mix(&o.tt_rank_max, sizeof(int32_t));
  mix(&o.aca_tol, sizeof(double));
  mix(&o.aca_rank_max, sizeof(int32_t));
  mix(&o.seed, sizeof(o.seed));
  mix(&o.quad_far_vol, sizeof(int32_t));
  mix(&o.quad_far_surf, sizeof(int32_t));
  return h;
}

int vsie_create(const vsie_problem* p, const vsie_options* opts, void* stream, vsie_handle** out) {
  return create_impl(p, opts, stream, nullptr, out);
}

int vsie_create_shared(const vsie_problem* p, const vsie_options* opts, vsie_handle* donor, void* stream,
                       vsie_handle** out) {
  if (!donor) return fail(VSIE_E_ARG, "null donor");
  if (!donor->H.far_share) return fail(VSIE_E_STATE, "the donor has no dense far block");
  return create_impl(p, opts, stream, donor, out);
}

static int create_impl(const vsie_problem* p, const vsie_options* opts, void* stream, vsie_handle* donor,
                       vsie_handle** out) {
  if (!p || !out) return fail(VSIE_E_ARG, "null argument");
  *out = nullptr;
  vsie_handle* hd = new (std::nothrow) vsie_handle();
  if (!hd) return fail(VSIE_E_NOMEM, "handle allocation");
  int rc = guarded([&]() {
    auto t0 = std::chrono::steady_clock::now();
    Handle& H = hd->H;
    if (opts) H.opts = *opts;
    else vsie_default_options(&H.opts);
    H.stream = (hipStream_t)stream;
    for (int a = 0; a < 3; ++a) {
      if (p->n[a] <= 0 || p->n[a] > 4096) throw Error(VSIE_E_ARG, "grid size out of range");
      H.n[a] = p->n[a];
      H.origin[a] = p->origin[a];
      if (!std::isfinite(p->origin[a])) throw Error(VSIE_E_ARG, "non-finite origin");
    }
    if (!(p->h > 0) || !std::isfinite(p->h)) throw Error(VSIE_E_ARG, "voxel size must be positive");
    if (!(p->freq_hz > 0) || !std::isfinite(p->freq_hz)) throw Error(VSIE_E_ARG, "frequency must be positive");
    if (!p->eps_r || !p->sigma) throw Error(VSIE_E_ARG, "null material arrays");
    if (H.opts.precorrect_dist < 0 || H.opts.tt_rank_max < 1 || H.opts.tt_rank_max > 128 ||
        H.opts.aca_rank_max < 1 || H.opts.aca_rank_max > 256 || !(H.opts.tt_tol > 0) || !(H.opts.aca_tol > 0) ||
        (H.opts.precision != VSIE_PREC_FP64 && H.opts.precision != VSIE_PREC_MIXED))
      throw Error(VSIE_E_ARG, "invalid options");
    if (H.opts.basis == VSIE_BASIS_PWL)
      throw Error(VSIE_E_UNSUPPORTED, "piecewise-linear body basis is not built (PWC only)");
    if (H.opts.basis != VSIE_BASIS_PWC) throw Error(VSIE_E_ARG, "unknown basis");
    if (H.opts.stencil != 5) throw Error(VSIE_E_UNSUPPORTED, "pFFT stencil: 5x5x5 blocks only");
    if (H.opts.quad_near_vol != 8 || H.opts.quad_near_surf != 5 || H.opts.quad_far_vol != 1 ||
        H.opts.quad_far_surf != 1)
      throw Error(VSIE_E_UNSUPPORTED, "coupling quadrature: 8 x 5 points near and 1 x 1 far only");
    if (p->n_meshes < 0 || (p->n_meshes > 0 && !p->meshes)) throw Error(VSIE_E_ARG, "bad mesh list");
    H.input_hash = input_hash(p, H.opts);
    H.h = p->h;
    H.freq = p->freq_hz;
    H.omega = 2.0 * PI * H.freq;
    H.k0 = H.omega * sqrt(EPS0 * MU0);
    H.nv = H.n[0] * H.n[1] * H.n[2];
    H.chi.resize(H.nv);
    for (int i = 0; i < H.nv; ++i) {
      double e = p->eps_r[i], s = p->sigma[i];
      if (!std::isfinite(e) || !std::isfinite(s)) throw Error(VSIE_E_ARG, "non-finite eps_r or sigma");
      H.chi[i] = cxd{e - 1.0, -s / (H.omega * EPS0)};
      if (H.chi[i].re != 0 || H.chi[i].im != 0) H.tissue.push_back(i);
    }
    std::vector<std::pair<int, std::vector<PortEdge>>> pf, pn;
    build_rwg(p, VSIE_FAR, H.far, pf);
    build_rwg(p, VSIE_NEAR, H.near, pn);
    H.mf = H.far.m;
    H.mn = H.near.m;
    if (donor) {
      if (H.mf == 0 || !donor->H.far_share->same(H.far, H.k0))
        throw Error(VSIE_E_ARG, "far conductors or frequency differ from the donor's");
      H.far_share = donor->H.far_share;
    }
    // ports in the order of the mesh list
    for (int mi = 0; mi < p->n_meshes; ++mi) {
      for (auto& q : pf)
        if (q.first == mi) H.ports.push_back(q.second);
      for (auto& q : pn)
        if (q.first == mi) H.ports.push_back(q.second);
    }
    H.N = (int64_t)H.mf + H.mn + 3LL * H.nv;
    if (H.mn > 0) stencil_setup(H);
    else {
      for (int a = 0; a < 3; ++a) {
        H.ne[a] = H.n[a];
        H.ob[a] = 0;
        int P = 8;
        while (P < 2 * H.ne[a] - 1) P *= 2;
        if (P > 1024) throw Error(VSIE_E_GRID, "grid needs an FFT longer than 1024");
        H.P[a] = P;
      }
      H.Ne = (int64_t)H.ne[0] * H.ne[1] * H.ne[2];
    }
    H.have32 = H.opts.precision != 0;
    progress("geometry and stencils", t0);
    {
      // delta-gap tables (Sec. II-A): b_m = s_m i w eps0 V0 l_m, V0 = 1 V
      const double ws = H.omega * EPS0;
      std::vector<int> idx;
      std::vector<double> vre, vim;
      H.port_off.assign(1, 0);
      for (const auto& pe : H.ports) {
        for (const PortEdge& e : pe) {
          const Rwg& R = e.domain == VSIE_FAR ? H.far : H.near;
          idx.push_back((e.domain == VSIE_FAR ? 0 : H.mf) + e.idx);
          vre.push_back(0.0);
          vim.push_back(ws * R.len[e.idx] * e.sign);
        }
        H.port_off.push_back((int)idx.size());
      }
      H.d_port_idx = upload(H, idx);
      H.d_port_re = upload(H, vre);
      H.d_port_im = upload(H, vim);
    }
    H.dfar = make_rwg_dev(H, H.far);
    H.dnear = make_rwg_dev(H, H.near);
    setup_volume(H);
    progress("generator and circulant spectra", t0);
    if (H.mn > 0) setup_pfft(H);
    progress("pFFT projection and precorrection", t0);
    if (H.mf > 0) {
      setup_dense_far(H);
      if (H.opts.precision) copy_zff_c64(H);
      progress("dense far block", t0);
      if (H.opts.build_far) {
        if (H.mn > 0) setup_aca(H);
        upload_aca(H);
        progress("ACA", t0);
        setup_tt(H);
        for (int chi = 0; chi < 3; ++chi) upload_tt(H, chi);
        progress("TT-cross", t0);
      }
    }
    alloc_work<double>(H, H.d64);
    if (H.opts.precision) alloc_work<float>(H, H.d32);
    tune_zpass<double>(H, H.d64);
    if (H.opts.precision) tune_zpass<float>(H, H.d32);
    VSIE_HIP(hipStreamSynchronize(H.stream));
    H.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
  if (rc != VSIE_OK) {
    delete hd;
    return rc;
  }
  *out = hd;
  return VSIE_OK;
}

int vsie_sizes(const vsie_handle* hd, vsie_sizes_t* s) {
  if (!hd || !s) return fail(VSIE_E_ARG, "null argument");
  const Handle& H = hd->H;
  std::memset(s, 0, sizeof(*s));
  s->n_total = H.N;
  s->m_far = H.mf;
  s->m_near = H.mn;
  for (int a = 0; a < 3; ++a) {
    s->n[a] = H.n[a];
    s->n_ext[a] = H.ne[a];
    s->fft[a] = H.P[a];
    s->tt_err_est[a] = H.tt_err[a];
    for (int k = 0; k < 3; ++k) s->tt_rank[a][k] = H.tt_r[a][k];
  }
  s->n_ports = (int)H.ports.size();
  s->n_tissue = (int)H.tissue.size();
  s->aca_rank = H.aca_k;
  s->precorr_nnz = H.pc_nnz;
  s->device_bytes = H.device_bytes;
  s->setup_seconds = H.setup_seconds;
  return VSIE_OK;
}

int vsie_rhs(const vsie_handle* hd, int port, int dtype, void* b_dev, void* stream) {
  if (!hd || !b_dev) return fail(VSIE_E_ARG, "null argument");
  const Handle& H = hd->H;
  if (port < 0 || port >= (int)H.ports.size()) return fail(VSIE_E_ARG, "port out of range");
  if (dtype != VSIE_C128 && dtype != VSIE_C64) return fail(VSIE_E_ARG, "bad dtype");
  return guarded([&]() {
    port_rhs(H, port, dtype, b_dev, (hipStream_t)stream);
    VSIE_HIP(hipGetLastError());
  });
}

int vsie_matvec(vsie_handle* hd, int dtype, int nrhs, const void* x_dev, void* y_dev, void* stream) {
  if (!hd || !x_dev || !y_dev || nrhs < 1) return fail(VSIE_E_ARG, "bad argument");
  if (x_dev == y_dev) return fail(VSIE_E_ARG, "x and y must not alias");
  Handle& H = hd->H;
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    if (dtype == VSIE_C128) {
      matvec_batch<double>(H, H.d64, (const cxd*)x_dev, (cxd*)y_dev, nrhs, st);
    } else if (dtype == VSIE_C64) {
      if (!H.have32) throw Error(VSIE_E_STATE, "complex64 operator data not built");
      matvec_batch<float>(H, H.d32, (const cxf*)x_dev, (cxf*)y_dev, nrhs, st);
    } else {
      throw Error(VSIE_E_ARG, "bad dtype");
    }
    VSIE_HIP(hipGetLastError());
  });
}

// Graph-replayed product: the launches of one vsie_matvec on fixed buffers, captured once on a
// capture stream (far-block chain on the same stream, no stage events) and replayed on the
// caller's stream. The product path makes no allocation, copy, fill or synchronisation; the only
// lazily allocated buffer (multi-column partial sums) is allocated before the capture.
static constexpr size_t GRAPH_CACHE = 16;
int vsie_matvec_graph(vsie_handle* hd, int dtype, int nrhs, const void* x_dev, void* y_dev, void* stream) {
  if (!hd || !x_dev || !y_dev || nrhs < 1) return fail(VSIE_E_ARG, "bad argument");
  if (x_dev == y_dev) return fail(VSIE_E_ARG, "x and y must not alias");
  if (dtype != VSIE_C128 && dtype != VSIE_C64) return fail(VSIE_E_ARG, "bad dtype");
  Handle& H = hd->H;
  if (dtype == VSIE_C64 && !H.have32) return fail(VSIE_E_STATE, "complex64 operator data not built");
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    Handle::GraphEntry* ge = nullptr;
    for (auto& g : H.graphs)
      if (g.dtype == dtype && g.nrhs == nrhs && g.x == x_dev && g.y == y_dev) ge = &g;
    if (!ge) {
      if (!H.gstream) VSIE_HIP(hipStreamCreateWithFlags(&H.gstream, hipStreamNonBlocking));
      auto prepare = [&](auto& D, auto zero) {
        using R = decltype(zero);
        if (nrhs > 1 && H.mf > 0 && !D.multi_part) {
          const int64_t nt = (int64_t)H.sym_T * (H.sym_T + 1) / 2;
          D.multi_part = H.dalloc<cx<R>>(16 * nt * 2 * SYM_TB);
        }
      };
      if (dtype == VSIE_C128) prepare(H.d64, 0.0);
      else prepare(H.d32, 0.0f);
      VSIE_HIP(hipStreamSynchronize(st));   // the capture stream must not overtake earlier work
      const bool conc = H.concurrent, prof = H.prof;
      H.concurrent = false;
      H.prof = false;
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(H.gstream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          if (dtype == VSIE_C128) matvec_batch<double>(H, H.d64, (const cxd*)x_dev, (cxd*)y_dev, nrhs, H.gstream);
          else matvec_batch<float>(H, H.d32, (const cxf*)x_dev, (cxf*)y_dev, nrhs, H.gstream);
        } catch (...) {
          (void)hipStreamEndCapture(H.gstream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          H.concurrent = conc;
          H.prof = prof;
          throw;
        }
        e = hipStreamEndCapture(H.gstream, &graph);
      }
      H.concurrent = conc;
      H.prof = prof;
      if (e != hipSuccess) throw Error(VSIE_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) throw Error(VSIE_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
      if (H.graphs.size() == GRAPH_CACHE) {
        (void)hipGraphExecDestroy(H.graphs.front().exec);
        H.graphs.erase(H.graphs.begin());
      }
      H.graphs.push_back(Handle::GraphEntry{dtype, nrhs, x_dev, y_dev, exec});
      ge = &H.graphs.back();
    }
    VSIE_HIP(hipGraphLaunch(ge->exec, st));
  });
}

// Products of several operators (phantoms of any grid sizes) captured one after another into one
// HIP graph, replayed by one launch.
int vsie_graph_create(int n, vsie_handle* const* hs, int dtype, const int* nrhs, const void* const* x,
                      void* const* y, void* stream, vsie_graph** out) {
  if (!out) return fail(VSIE_E_ARG, "null argument");
  *out = nullptr;
  if (n < 1 || !hs || !nrhs || !x || !y) return fail(VSIE_E_ARG, "bad argument");
  if (dtype != VSIE_C128 && dtype != VSIE_C64) return fail(VSIE_E_ARG, "bad dtype");
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !x[i] || !y[i] || nrhs[i] < 1 || x[i] == y[i]) return fail(VSIE_E_ARG, "bad operator or buffer");
    if (dtype == VSIE_C64 && !hs[i]->H.have32) return fail(VSIE_E_STATE, "complex64 operator data not built");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(VSIE_E_ARG, "an operator appears twice (its work buffers are shared)");
  }
  vsie_graph* g = new (std::nothrow) vsie_graph();
  if (!g) return fail(VSIE_E_NOMEM, "graph allocation");
  const int rc = guarded([&]() {
    VSIE_HIP(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    for (int i = 0; i < n; ++i) {
      Handle& H = hs[i]->H;
      if (nrhs[i] > 1 && H.mf > 0) {
        const int64_t nt = (int64_t)H.sym_T * (H.sym_T + 1) / 2;
        if (dtype == VSIE_C128 && !H.d64.multi_part) H.d64.multi_part = H.dalloc<cxd>(16 * nt * 2 * SYM_TB);
        if (dtype == VSIE_C64 && !H.d32.multi_part) H.d32.multi_part = H.dalloc<cxf>(16 * nt * 2 * SYM_TB);
      }
    }
    VSIE_HIP(hipStreamSynchronize((hipStream_t)stream));
    std::vector<std::pair<bool, bool>> saved;
    for (int i = 0; i < n; ++i) {
      saved.push_back({hs[i]->H.concurrent, hs[i]->H.prof});
      hs[i]->H.concurrent = false;
      hs[i]->H.prof = false;
    }
    auto restore = [&]() {
      for (int i = 0; i < n; ++i) {
        hs[i]->H.concurrent = saved[i].first;
        hs[i]->H.prof = saved[i].second;
      }
    };
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        for (int i = 0; i < n; ++i) {
          Handle& H = hs[i]->H;
          if (dtype == VSIE_C128) matvec_batch<double>(H, H.d64, (const cxd*)x[i], (cxd*)y[i], nrhs[i], g->cap);
          else matvec_batch<float>(H, H.d32, (const cxf*)x[i], (cxf*)y[i], nrhs[i], g->cap);
        }
      } catch (...) {
        (void)hipStreamEndCapture(g->cap, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        restore();
        throw;
      }
      e = hipStreamEndCapture(g->cap, &graph);
    }
    restore();
    if (e != hipSuccess) throw Error(VSIE_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) throw Error(VSIE_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
  });
  if (rc != VSIE_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
    return rc;
  }
  *out = g;
  return VSIE_OK;
}

int vsie_graph_launch(vsie_graph* g, void* stream) {
  if (!g || !g->exec) return fail(VSIE_E_ARG, "null graph");
  return guarded([&]() { VSIE_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream)); });
}

int vsie_graph_destroy(vsie_graph* g) {
  if (!g) return VSIE_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  delete g;
  return VSIE_OK;
}

// Checkpoint file: "VSIECKPT", uint32 version, uint64 input hash, uint32 records, then per record
// uint32 kind, uint32 index, uint64 bytes and the vsie_export bytes of that record.
static const char CKPT_MAGIC[8] = {'V', 'S', 'I', 'E', 'C', 'K', 'P', 'T'};
static constexpr uint32_t CKPT_VERSION = 1;

// the checks vsie_import makes of a record's kind, index, ranks and size, made before any import
static bool checkpoint_record_ok(const Handle& H, uint32_t what, uint32_t index, const std::vector<unsigned char>& b) {
  if (what == VSIE_X_TT_CORES) {
    if (index > 2 || H.mf == 0 || b.size() < 3 * sizeof(int)) return false;
    int r[3];
    std::memcpy(r, b.data(), sizeof(r));
    for (int k = 0; k < 3; ++k)
      if (r[k] < 1 || r[k] > 128) return false;
    const size_t n = (size_t)H.n[0] * r[0] + (size_t)r[0] * H.n[1] * r[1] + (size_t)r[1] * H.n[2] * r[2] +
                     (size_t)r[2] * H.mf;
    return b.size() == 3 * sizeof(int) + sizeof(cxd) * n;
  }
  if (what == VSIE_X_ACA) {
    if (index != 0 || H.mf == 0 || H.mn == 0 || b.size() < sizeof(int)) return false;
    int k;
    std::memcpy(&k, b.data(), sizeof(int));
    return k >= 0 && k <= 256 && b.size() == sizeof(int) + sizeof(cxd) * ((size_t)H.mn * k + (size_t)H.mf * k);
  }
  return false;
}

int vsie_checkpoint_save(const vsie_handle* hd, const char* path) {
  if (!hd || !path) return fail(VSIE_E_ARG, "null argument");
  const Handle& H = hd->H;
  if (H.mf == 0) return fail(VSIE_E_STATE, "no far conductors: nothing to checkpoint");
  return guarded([&]() {
    std::vector<std::pair<std::pair<uint32_t, uint32_t>, std::vector<unsigned char>>> recs;
    auto add = [&](int what, int index) {
      size_t n = 0;
      if (vsie_export(hd, what, index, nullptr, &n) != VSIE_OK) throw Error(VSIE_E_STATE, "export failed");
      std::vector<unsigned char> b(n);
      if (vsie_export(hd, what, index, b.data(), &n) != VSIE_OK) throw Error(VSIE_E_STATE, "export failed");
      recs.push_back({{(uint32_t)what, (uint32_t)index}, std::move(b)});
    };
    for (int c = 0; c < 3; ++c)
      if (!H.tt_host[c][0].empty()) add(VSIE_X_TT_CORES, c);
    if (H.mn > 0 && H.aca_k > 0) add(VSIE_X_ACA, 0);
    const std::string tmp = std::string(path) + ".part";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) throw Error(VSIE_E_ARG, std::string("cannot write ") + tmp);
    bool ok = std::fwrite(CKPT_MAGIC, 1, 8, f) == 8;
    const uint32_t ver = CKPT_VERSION, nrec = (uint32_t)recs.size();
    ok = ok && std::fwrite(&ver, 4, 1, f) == 1 && std::fwrite(&H.input_hash, 8, 1, f) == 1 &&
         std::fwrite(&nrec, 4, 1, f) == 1;
    for (const auto& r : recs) {
      const uint64_t nb = r.second.size();
      ok = ok && std::fwrite(&r.first.first, 4, 1, f) == 1 && std::fwrite(&r.first.second, 4, 1, f) == 1 &&
           std::fwrite(&nb, 8, 1, f) == 1 && std::fwrite(r.second.data(), 1, nb, f) == nb;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
      std::remove(tmp.c_str());
      throw Error(VSIE_E_ARG, std::string("cannot write ") + path);
    }
  });
}

int vsie_checkpoint_load(vsie_handle* hd, const char* path) {
  if (!hd || !path) return fail(VSIE_E_ARG, "null argument");
  Handle& H = hd->H;
  if (H.schur.ready) return fail(VSIE_E_STATE, "the far elimination was built from the current factors");
  return guarded([&]() {
    FILE* f = std::fopen(path, "rb");
    if (!f) throw Error(VSIE_E_ARG, std::string("cannot read ") + path);
    struct Closer {
      FILE* f;
      ~Closer() { std::fclose(f); }
    } closer{f};
    // bytes in the file, so that a damaged record length is refused before anything is allocated
    if (std::fseek(f, 0, SEEK_END) != 0) throw Error(VSIE_E_ARG, std::string("cannot read ") + path);
    const long fsize = std::ftell(f);
    if (fsize < 0 || std::fseek(f, 0, SEEK_SET) != 0) throw Error(VSIE_E_ARG, std::string("cannot read ") + path);
    const uint64_t total = (uint64_t)fsize;
    char magic[8];
    uint32_t ver = 0, nrec = 0;
    uint64_t hash = 0;
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, CKPT_MAGIC, 8) != 0)
      throw Error(VSIE_E_ARG, "not a checkpoint file");
    if (std::fread(&ver, 4, 1, f) != 1 || ver != CKPT_VERSION) throw Error(VSIE_E_ARG, "checkpoint version differs");
    if (std::fread(&hash, 8, 1, f) != 1 || hash != H.input_hash)
      throw Error(VSIE_E_ARG, "checkpoint was written for other inputs or compression options");
    if (std::fread(&nrec, 4, 1, f) != 1 || nrec > 16) throw Error(VSIE_E_ARG, "corrupt checkpoint");
    // read every record before importing any, so that a damaged file changes nothing
    std::vector<std::pair<std::pair<uint32_t, uint32_t>, std::vector<unsigned char>>> recs;
    for (uint32_t i = 0; i < nrec; ++i) {
      uint32_t what = 0, index = 0;
      uint64_t nb = 0;
      if (std::fread(&what, 4, 1, f) != 1 || std::fread(&index, 4, 1, f) != 1 || std::fread(&nb, 8, 1, f) != 1)
        throw Error(VSIE_E_ARG, "truncated checkpoint");
      const long pos = std::ftell(f);
      if (pos < 0 || (uint64_t)pos > total || nb > total - (uint64_t)pos)
        throw Error(VSIE_E_ARG, "truncated checkpoint");
      std::vector<unsigned char> b(nb);
      if (std::fread(b.data(), 1, nb, f) != nb) throw Error(VSIE_E_ARG, "truncated checkpoint");
      if (!checkpoint_record_ok(H, what, index, b)) throw Error(VSIE_E_ARG, "corrupt checkpoint");
      recs.push_back({{what, index}, std::move(b)});
    }
    for (const auto& r : recs) {
      const int rc = vsie_import(hd, (int)r.first.first, (int)r.first.second, r.second.data(), r.second.size());
      if (rc != VSIE_OK) throw Error(rc, std::string("checkpoint record rejected: ") + vsie_last_error());
    }
  });
}

int vsie_zpass_tuning(vsie_handle* hd, int dtype, int* chosen, int* v, int* np, double* ms) {
  if (!hd || !chosen || !v || !np || !ms) return fail(VSIE_E_ARG, "null argument");
  if (dtype != VSIE_C128 && dtype != VSIE_C64) return fail(VSIE_E_ARG, "bad dtype");
  Handle& H = hd->H;
  const int p = dtype == VSIE_C128 ? 0 : 1;
  if (p == 1 && !H.have32) return fail(VSIE_E_STATE, "complex64 operator data not built");
  return guarded([&]() {
    *chosen = H.zcand[p];
    for (int c = 0; c < 3; ++c) {
      zconv_shape(H.P[2], p == 0, c, &v[c], &np[c]);
      ms[c] = H.ztime[p][c];
    }
  });
}

int vsie_zpass_select(vsie_handle* hd, int dtype, int cand) {
  if (!hd) return fail(VSIE_E_ARG, "null argument");
  if (dtype != VSIE_C128 && dtype != VSIE_C64) return fail(VSIE_E_ARG, "bad dtype");
  Handle& H = hd->H;
  const int p = dtype == VSIE_C128 ? 0 : 1;
  if (p == 1 && !H.have32) return fail(VSIE_E_STATE, "complex64 operator data not built");
  if (H.P[2] < 64 || H.P[2] > 1024) return fail(VSIE_E_STATE, "this grid's z pass has no candidates");
  if (!zconv_candidate(H.P[2], p == 0, cand)) return fail(VSIE_E_ARG, "no such z-pass candidate for this length");
  return guarded([&]() {
    VSIE_HIP(hipStreamSynchronize(H.stream));
    H.d_zorder[p] = upload<int>(H, zconv_order(H.P[2], H.P[0], H.P[1], p == 0, cand));
    H.zcand[p] = cand;
    for (auto& g : H.graphs) (void)hipGraphExecDestroy(g.exec);
    H.graphs.clear();
  });
}

static int check_solve_opts(const vsie_handle* hd, const vsie_solve_opts* o, vsie_solve_opts& so) {
  if (o) so = *o;
  else vsie_default_solve_opts(&so);
  if (so.restart < 1 || so.restart > 1000 || so.max_iter < 1 || !(so.tol > 0)) return fail(VSIE_E_ARG, "bad solve options");
  if (so.method < VSIE_GMRES64 || so.method > VSIE_SCHUR_LEARNED) return fail(VSIE_E_ARG, "unknown solve method");
  if (so.method == VSIE_SCHUR_LEARNED && !hd->H.net) return fail(VSIE_E_STATE, "no network attached (vsie_net_attach)");
  if (!(so.reorth >= 0 && so.reorth <= 1)) return fail(VSIE_E_ARG, "reorth must lie in [0, 1]");
  if ((so.method == VSIE_IR_MIXED || so.method == VSIE_SCHUR_MIXED) && !hd->H.have32)
    return fail(VSIE_E_STATE, "complex64 operator data not built");
  return VSIE_OK;
}

static int solve_impl(vsie_handle* hd, const vsie_solve_opts& so, int nrhs, const void* b_dev, void* x_dev,
                      vsie_solve_stats* stats, void* stream);

int vsie_solve(vsie_handle* hd, const vsie_solve_opts* o, int nrhs, const void* b_dev, void* x_dev,
               vsie_solve_stats* stats, void* stream) {
  if (!hd || !b_dev || !x_dev || nrhs < 1) return fail(VSIE_E_ARG, "bad argument");
  vsie_solve_opts so;
  const int rc = check_solve_opts(hd, o, so);
  if (rc != VSIE_OK) return rc;
  return solve_impl(hd, so, nrhs, b_dev, x_dev, stats, stream);
}

int vsie_solve_ports(vsie_handle* hd, const vsie_solve_opts* o, int nports, const int32_t* ports, void* x_dev,
                     vsie_solve_stats* stats, void* stream) {
  if (!hd || !ports || !x_dev || nports < 1) return fail(VSIE_E_ARG, "bad argument");
  for (int i = 0; i < nports; ++i)
    if (ports[i] < 0 || ports[i] >= (int)hd->H.ports.size()) return fail(VSIE_E_ARG, "port out of range");
  vsie_solve_opts so;
  int rc = check_solve_opts(hd, o, so);
  if (rc != VSIE_OK) return rc;
  void* b = nullptr;
  rc = guarded([&]() {
    const size_t bytes = sizeof(cxd) * (size_t)hd->H.N * nports;
    if (hipMalloc(&b, bytes) != hipSuccess) {
      b = nullptr;
      throw Error(VSIE_E_NOMEM, "hipMalloc of the port right-hand sides failed");
    }
    for (int i = 0; i < nports; ++i) port_rhs(hd->H, ports[i], VSIE_C128, (cxd*)b + (size_t)i * hd->H.N, (hipStream_t)stream);
    VSIE_HIP(hipGetLastError());
  });
  if (rc == VSIE_OK) rc = solve_impl(hd, so, nports, b, x_dev, stats, stream);
  if (b) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(b);
  }
  return rc;
}

static int solve_impl(vsie_handle* hd, const vsie_solve_opts& so, int nrhs, const void* b_dev, void* x_dev,
                      vsie_solve_stats* stats, void* stream) {
  Handle& H = hd->H;
  int status = VSIE_OK;
  int rc = guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    ensure_solver_ws(H, so.restart);
    // Krylov work runs on the compact vector of coupled unknowns (conductor currents and tissue
    // voxels; air voxels decouple with identity rows and columns and take x = b); products
    // scatter into and gather from full-length vectors
    const int64_t N = H.N, Nc = H.n_active;
    const bool mixed = so.method == VSIE_IR_MIXED || so.method == VSIE_SCHUR_MIXED;
    std::vector<Scratch> bufs;
    auto vec = [&](int64_t n, size_t elem) { bufs.emplace_back(elem * (size_t)n); return bufs.back().p; };
    bufs.reserve(12);
    SolveWork ws{};
    ws.wc = (cxd*)vec(Nc, sizeof(cxd));
    ws.bc = (cxd*)vec(Nc, sizeof(cxd));
    ws.xc = (cxd*)vec(Nc, sizeof(cxd));
    ws.dc = (cxd*)vec(Nc, sizeof(cxd));
    cxd* r = (cxd*)vec(N, sizeof(cxd));
    ws.hv = (cxd*)vec(1100, sizeof(cxd));
    if (mixed) {
      ws.x32 = (cxf*)vec(N, sizeof(cxf));
      ws.y32 = (cxf*)vec(N, sizeof(cxf));
      ws.Vout = (cxd*)vec(Nc * (IR_OUTER_M + 1), sizeof(cxd));
      ws.Zout = (cxd*)vec(Nc * IR_OUTER_M, sizeof(cxd));
      ws.hv2 = (cxd*)vec(1100, sizeof(cxd));
    }
    cxd *wc = ws.wc, *bc = ws.bc, *xc = ws.xc, *dc = ws.dc, *hv = ws.hv, *hv2 = ws.hv2, *Vout = ws.Vout,
        *Zout = ws.Zout;
    cxf *x32 = ws.x32, *y32 = ws.y32;
    cxd* fin = H.d_full[0];
    cxd* fout = H.d_full[1];
    Solver S(H, st);
    S.kappa = so.reorth;
    auto A64 = [&](const cxd* in, cxd* out) {
      launch_scatter_idx(st, in, H.d_active, Nc, fin);
      matvec_one<double>(H, H.d64, fin, fout, st);
      launch_gather_idx(st, fout, H.d_active, Nc, out);
    };
    auto A32 = [&](const cxd* in, cxd* out) {
      launch_scatter_idx(st, in, H.d_active, Nc, fin);
      launch_d2f(st, fin, x32, N);
      matvec_one<float>(H, H.d32, x32, y32, st);
      launch_f2d(st, y32, fout, N);
      launch_gather_idx(st, fout, H.d_active, Nc, out);
    };
    const bool schur = so.method == VSIE_SCHUR || so.method == VSIE_SCHUR_MIXED || so.method == VSIE_SCHUR_LEARNED;
    if (schur) setup_schur(H, so.precond != 0 || so.method == VSIE_SCHUR_LEARNED);
    if (so.method == VSIE_SCHUR_LEARNED) {
      ws.Vout = (cxd*)vec(Nc * (so.restart + 1), sizeof(cxd));
      ws.Zout = (cxd*)vec(Nc * so.restart, sizeof(cxd));
    }
    for (int c = 0; c < nrhs; ++c) {
      auto t0 = std::chrono::steady_clock::now();
      const cxd* b = (const cxd*)b_dev + c * N;
      cxd* x = (cxd*)x_dev + c * N;
      vsie_solve_stats s;
      std::memset(&s, 0, sizeof(s));
      const int64_t passes0 = S.second_passes;
      double rel = 0;
      if (schur) {
        s.iterations = solve_schur(H, S, so, so.method == VSIE_SCHUR_MIXED, b, x, ws, &s.restarts, &s.refinements, &rel,
                                   st);
      } else {
        launch_gather_idx(st, b, H.d_active, Nc, bc);
        if (so.method == VSIE_GMRES64) {
          s.iterations = S.gmres(A64, bc, xc, so.tol, so.restart, so.max_iter, &s.restarts, &rel, H.d_krylov, wc, hv);
        } else {
          int total = 0;
          // preconditioner: at most one cycle (restart iterations) of complex64 GMRES on Z z = v
          auto P32 = [&](const cxd* v, cxd* z) {
            double inner_rel = 0;
            int used = S.gmres(A32, v, z, so.inner_tol, so.restart,
                               std::max(1, std::min(so.restart, so.max_iter - total)), &s.restarts, &inner_rel,
                               H.d_krylov, dc, hv2);
            total += used;
            return total < so.max_iter;
          };
          S.fgmres(A64, P32, bc, xc, so.tol, IR_OUTER_M, &s.refinements, &rel, Vout, Zout, wc, hv);
          s.iterations = total;
        }
        VSIE_HIP(hipMemcpyAsync(x, b, sizeof(cxd) * N, hipMemcpyDeviceToDevice, st));
        launch_scatter_idx(st, xc, H.d_active, Nc, x);
      }
      // true FP64 residual of the full system and per-block residuals
      matvec_one<double>(H, H.d64, x, fout, st);
      launch_sub(st, b, fout, r, N);
      double nr[4], nb[4];
      S.norms(r, nr, N);
      S.norms(b, nb, N);
      s.rel_residual = nb[3] > 0 ? nr[3] / nb[3] : 0;
      for (int q = 0; q < 3; ++q) s.block_residual[q] = nb[3] > 0 ? nr[q] / nb[3] : 0;
      VSIE_HIP(hipStreamSynchronize(st));
      s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      s.gs_second_passes = (int32_t)(S.second_passes - passes0);
      if (s.rel_residual > so.tol) status = VSIE_E_NOCONV;
      if (stats) stats[c] = s;
    }
    VSIE_HIP(hipStreamSynchronize(st));
  });
  if (rc != VSIE_OK) return rc;
  if (status != VSIE_OK) return fail(status, "solver did not reach the requested tolerance");
  return VSIE_OK;
}

int vsie_port_current(const vsie_handle* hd, int port, const double* x, double* I) {
  if (!hd || !x || !I) return fail(VSIE_E_ARG, "null argument");
  const Handle& H = hd->H;
  if (port < 0 || port >= (int)H.ports.size()) return fail(VSIE_E_ARG, "port out of range");
  double re = 0, im = 0;
  for (const PortEdge& e : H.ports[port]) {
    const Rwg& R = e.domain == VSIE_FAR ? H.far : H.near;
    int64_t g = (e.domain == VSIE_FAR ? 0 : H.mf) + e.idx;
    re += e.sign * R.len[e.idx] * x[2 * g];
    im += e.sign * R.len[e.idx] * x[2 * g + 1];
  }
  I[0] = re;
  I[1] = im;
  return VSIE_OK;
}

int vsie_export(const vsie_handle* hd, int what, int index, void* host, size_t* nbytes) {
  if (!hd || !nbytes) return fail(VSIE_E_ARG, "null argument");
  const Handle& H = hd->H;
  return guarded([&]() {
    std::vector<unsigned char> buf;
    auto put = [&](const void* p, size_t n) {
      const unsigned char* c = (const unsigned char*)p;
      buf.insert(buf.end(), c, c + n);
    };
    switch (what) {
      case VSIE_X_TT_CORES: {
        if (index < 0 || index > 2) throw Error(VSIE_E_ARG, "TT component out of range");
        put(H.tt_r[index], sizeof(int) * 3);
        for (int k = 0; k < 4; ++k) put(H.tt_host[index][k].data(), sizeof(cxd) * H.tt_host[index][k].size());
        break;
      }
      case VSIE_X_ACA: {
        put(&H.aca_k, sizeof(int));
        put(H.aca_U.data(), sizeof(cxd) * H.aca_U.size());
        put(H.aca_V.data(), sizeof(cxd) * H.aca_V.size());
        break;
      }
      case VSIE_X_STENCIL: {
        put(H.base.data(), sizeof(int) * H.base.size());
        put(H.Wh.data(), sizeof(double) * H.Wh.size());
        break;
      }
      case VSIE_X_GENERATOR: {
        std::vector<cxd> o = download(H.d_oct, 6 * H.Ne);
        put(o.data(), sizeof(cxd) * o.size());
        break;
      }
      case VSIE_X_EXT_GRID: {
        put(H.ne, sizeof(int) * 3);
        put(H.ob, sizeof(int) * 3);
        put(H.P, sizeof(int) * 3);
        break;
      }
      default:
        throw Error(VSIE_E_ARG, "unknown export kind");
    }
    if (!host) {
      *nbytes = buf.size();
      return;
    }
    if (*nbytes < buf.size()) throw Error(VSIE_E_ARG, "export buffer too small");
    std::memcpy(host, buf.data(), buf.size());
    *nbytes = buf.size();
  });
}

int vsie_import(vsie_handle* hd, int what, int index, const void* host, size_t nbytes) {
  if (!hd || !host) return fail(VSIE_E_ARG, "null argument");
  Handle& H = hd->H;
  if (H.schur.ready) return fail(VSIE_E_STATE, "the far elimination was built from the current factors");
  return guarded([&]() {
    // captured products hold the factors' device addresses: drop them
    VSIE_HIP(hipDeviceSynchronize());
    for (auto& g : H.graphs) (void)hipGraphExecDestroy(g.exec);
    H.graphs.clear();
    const unsigned char* c = (const unsigned char*)host;
    if (what == VSIE_X_TT_CORES) {
      if (index < 0 || index > 2) throw Error(VSIE_E_ARG, "TT component out of range");
      if (H.mf == 0) throw Error(VSIE_E_STATE, "no far conductors");
      if (nbytes < 3 * sizeof(int)) throw Error(VSIE_E_ARG, "short TT record");
      int r[3];
      std::memcpy(r, c, sizeof(r));
      for (int k = 0; k < 3; ++k)
        if (r[k] < 1 || r[k] > 128) throw Error(VSIE_E_ARG, "TT rank must be within 1..128");
      size_t sz[4] = {(size_t)H.n[0] * r[0], (size_t)r[0] * H.n[1] * r[1], (size_t)r[1] * H.n[2] * r[2],
                      (size_t)r[2] * H.mf};
      size_t need = 3 * sizeof(int) + sizeof(cxd) * (sz[0] + sz[1] + sz[2] + sz[3]);
      if (nbytes != need) throw Error(VSIE_E_ARG, "TT record size mismatch");
      size_t off = 3 * sizeof(int);
      for (int k = 0; k < 4; ++k) {
        H.tt_host[index][k].resize(sz[k]);
        std::memcpy(H.tt_host[index][k].data(), c + off, sizeof(cxd) * sz[k]);
        off += sizeof(cxd) * sz[k];
      }
      for (int k = 0; k < 3; ++k) H.tt_r[index][k] = r[k];
      H.tt_err[index] = 0;
      upload_tt(H, index);
    } else if (what == VSIE_X_ACA) {
      if (H.mf == 0 || H.mn == 0) throw Error(VSIE_E_STATE, "needs near and far conductors");
      int k;
      if (nbytes < sizeof(int)) throw Error(VSIE_E_ARG, "short ACA record");
      std::memcpy(&k, c, sizeof(int));
      if (k < 0 || k > 256) throw Error(VSIE_E_ARG, "ACA rank must be within 0..256");
      size_t need = sizeof(int) + sizeof(cxd) * ((size_t)H.mn * k + (size_t)H.mf * k);
      if (nbytes != need) throw Error(VSIE_E_ARG, "ACA record size mismatch");
      H.aca_k = k;
      H.aca_U.resize((size_t)H.mn * k);
      H.aca_V.resize((size_t)H.mf * k);
      std::memcpy(H.aca_U.data(), c + sizeof(int), sizeof(cxd) * H.aca_U.size());
      std::memcpy(H.aca_V.data(), c + sizeof(int) + sizeof(cxd) * H.aca_U.size(), sizeof(cxd) * H.aca_V.size());
      upload_aca(H);
    } else {
      throw Error(VSIE_E_ARG, "unsupported import kind");
    }
  });
}

int vsie_schur_setup(vsie_handle* hd, int precond) {
  if (!hd) return fail(VSIE_E_ARG, "null handle");
  Handle& H = hd->H;
  return guarded([&]() { setup_schur(H, precond != 0); });
}

int vsie_schur_info(const vsie_handle* hd, int32_t* n_proxy, double* seconds, int32_t* built) {
  if (!hd) return fail(VSIE_E_ARG, "null handle");
  const Handle::Schur& Sc = hd->H.schur;
  if (n_proxy) *n_proxy = Sc.K;
  if (seconds) *seconds = Sc.seconds;
  if (built) *built = (Sc.ready ? 1 : 0) | (Sc.precond ? 2 : 0);
  return VSIE_OK;
}

int vsie_schur_matvec(vsie_handle* hd, const void* x_dev, void* y_dev, void* stream) {
  if (!hd || !x_dev || !y_dev || x_dev == y_dev) return fail(VSIE_E_ARG, "bad argument");
  Handle& H = hd->H;
  if (!H.schur.ready) return fail(VSIE_E_STATE, "far elimination not set up (vsie_schur_setup)");
  return guarded([&]() {
    matvec_schur<double>(H, (const cxd*)x_dev, (cxd*)y_dev, (hipStream_t)stream);
    VSIE_HIP(hipGetLastError());
  });
}

int vsie_schur_precond(vsie_handle* hd, const void* x_dev, void* y_dev, void* stream) {
  if (!hd || !x_dev || !y_dev || x_dev == y_dev) return fail(VSIE_E_ARG, "bad argument");
  Handle& H = hd->H;
  if (!H.schur.precond) return fail(VSIE_E_STATE, "preconditioner not built (vsie_schur_setup with precond)");
  return guarded([&]() {
    precond_apply<double>(H, (const cxd*)x_dev, (cxd*)y_dev, (hipStream_t)stream);
    VSIE_HIP(hipGetLastError());
  });
}

int vsie_dense_lu_solve(int n, void* A_dev, int64_t lda, void* B_dev, int64_t ldb, int nrhs, void* stream) {
  if (n < 0 || nrhs < 0 || lda < n || ldb < nrhs || (n > 0 && (!A_dev || (nrhs > 0 && !B_dev))))
    return fail(VSIE_E_ARG, "bad argument");
  if (n == 0) return VSIE_OK;
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    DenseLU F;
    F.n = n;
    F.lda = lda;
    F.A = (cxd*)A_dev;
    Scratch Li(sizeof(cxd) * lu_blocks_elems(n)), Ui(sizeof(cxd) * lu_blocks_elems(n)), ip(sizeof(int) * n),
        pm(sizeof(int) * n), inf(sizeof(int)), work(sizeof(cxd) * lu_work_elems(n));
    F.Linv = Li.as<cxd>();
    F.Uinv = Ui.as<cxd>();
    F.d_ipiv = ip.as<int>();
    F.d_perm = pm.as<int>();
    F.d_info = inf.as<int>();
    lu_factor(st, F, work.as<cxd>());
    if (nrhs > 0) {
      Scratch W(sizeof(cxd) * (size_t)n * nrhs);
      lu_solve(st, F, (cxd*)B_dev, ldb, nrhs, W.as<cxd>());
      VSIE_HIP(hipStreamSynchronize(st));
    }
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Workspace of vsie_dense_lu_solve_noalloc: one static device array per GPU, carved into the
// inverted diagonal blocks, the factorisation's work panel, the solve's n x nrhs buffer, the pivots,
// the permutation and the singularity flag. Host code never passes the array's name to a kernel
// (on the host it only stands for the symbol): each device's address is looked up once with
// hipGetSymbolAddress and kept in g_lu_scratch_ptr.
namespace {
constexpr int64_t LU_NA_ALIGN = 256;
constexpr int64_t lu_na_round(int64_t b) { return (b + LU_NA_ALIGN - 1) / LU_NA_ALIGN * LU_NA_ALIGN; }
constexpr int64_t LU_NA_BLK = lu_na_round((int64_t)((VSIE_LU_NOALLOC_MAX_N + LU_NB - 1) / LU_NB) * LU_NB * LU_NB * 16);
constexpr int64_t LU_NA_WORK = lu_na_round((int64_t)LU_NB * VSIE_LU_NOALLOC_MAX_N * 16);
constexpr int64_t LU_NA_W = lu_na_round((int64_t)VSIE_LU_NOALLOC_MAX_N * VSIE_LU_NOALLOC_MAX_NRHS * 16);
constexpr int64_t LU_NA_INT = lu_na_round((int64_t)VSIE_LU_NOALLOC_MAX_N * 4);
constexpr int64_t LU_NA_BYTES = 2 * LU_NA_BLK + LU_NA_WORK + LU_NA_W + 2 * LU_NA_INT + LU_NA_ALIGN;
static_assert(VSIE_LU_NOALLOC_MAX_N <= LU_PERM_LDS, "permutation formed on the device");
constexpr int LU_NA_MAX_DEVICES = 64;
std::mutex g_lu_scratch_mutex;
void* g_lu_scratch_ptr[LU_NA_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[LU_NA_BYTES];

// device address of this GPU's copy of scratch (looked up on the first call on that device)
static void* lu_scratch_address() {
  int dev = 0;
  VSIE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= LU_NA_MAX_DEVICES) throw Error(VSIE_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_lu_scratch_mutex);
  if (!g_lu_scratch_ptr[dev]) {
    void* ptr = nullptr;
    VSIE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(VSIE_E_HIP, "hipGetSymbolAddress returned no address");
    g_lu_scratch_ptr[dev] = ptr;
  }
  return g_lu_scratch_ptr[dev];
}

extern "C" {

int vsie_dense_lu_solve_noalloc(int n, void* A_dev, int64_t lda, void* B_dev, int64_t ldb, int nrhs, void* stream) {
  if (n < 0 || nrhs < 0 || lda < n || ldb < nrhs || (n > 0 && (!A_dev || (nrhs > 0 && !B_dev))))
    return fail(VSIE_E_ARG, "bad argument");
  if (n > VSIE_LU_NOALLOC_MAX_N || nrhs > VSIE_LU_NOALLOC_MAX_NRHS)
    return fail(VSIE_E_ARG, "dense LU without allocation: n <= " + std::to_string(VSIE_LU_NOALLOC_MAX_N) +
                                " and nrhs <= " + std::to_string(VSIE_LU_NOALLOC_MAX_NRHS) + " only");
  if (n == 0) return VSIE_OK;
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    unsigned char* base = (unsigned char*)lu_scratch_address();
    DenseLU F;
    F.n = n;
    F.lda = lda;
    F.A = (cxd*)A_dev;
    F.Linv = (cxd*)base;
    F.Uinv = (cxd*)(base + LU_NA_BLK);
    cxd* work = (cxd*)(base + 2 * LU_NA_BLK);
    cxd* W = (cxd*)(base + 2 * LU_NA_BLK + LU_NA_WORK);
    F.d_ipiv = (int*)(base + 2 * LU_NA_BLK + LU_NA_WORK + LU_NA_W);
    F.d_perm = (int*)(base + 2 * LU_NA_BLK + LU_NA_WORK + LU_NA_W + LU_NA_INT);
    F.d_info = (int*)(base + 2 * LU_NA_BLK + LU_NA_WORK + LU_NA_W + 2 * LU_NA_INT);
    lu_factor(st, F, work, true);   // clears the flag, blocks to read it back
    if (nrhs > 0) {
      lu_solve(st, F, (cxd*)B_dev, ldb, nrhs, W);
      VSIE_HIP(hipStreamSynchronize(st));
    }
  });
}

// ---------------------------------------------------------------------------------------------
// learned preconditioner

int vsie_net_create(uint64_t seed, int64_t pair_capacity, vsie_net** out) {
  if (!out || pair_capacity < 0) return fail(VSIE_E_ARG, "bad argument");
  *out = nullptr;
  vsie_net* n = new (std::nothrow) vsie_net();
  if (!n) return fail(VSIE_E_NOMEM, "network allocation");
  int rc = guarded([&]() {
    cnn_init(n->S.N, seed);
    n->S.cap = pair_capacity;
  });
  if (rc != VSIE_OK) {
    delete n;
    return rc;
  }
  *out = n;
  return VSIE_OK;
}

void vsie_net_destroy(vsie_net* n) { delete n; }

int vsie_net_info(const vsie_net* n, int64_t* nparam, int64_t* n_pairs, int64_t* adam_steps) {
  if (!n) return fail(VSIE_E_ARG, "null network");
  if (nparam) *nparam = n->S.N.nparam;
  if (n_pairs) *n_pairs = n->S.count;
  if (adam_steps) *adam_steps = n->S.N.step;
  return VSIE_OK;
}

int vsie_net_get_params(const vsie_net* n, float* host, int64_t count) {
  if (!n || !host || count != n->S.N.nparam) return fail(VSIE_E_ARG, "bad argument");
  return guarded([&]() {
    VSIE_HIP(hipDeviceSynchronize());
    VSIE_HIP(hipMemcpy(host, n->S.N.params, sizeof(float) * count, hipMemcpyDeviceToHost));
  });
}

int vsie_net_set_params(vsie_net* n, const float* host, int64_t count) {
  if (!n || !host || count != n->S.N.nparam) return fail(VSIE_E_ARG, "bad argument");
  return guarded([&]() {
    VSIE_HIP(hipDeviceSynchronize());
    VSIE_HIP(hipMemcpy(n->S.N.params, host, sizeof(float) * count, hipMemcpyHostToDevice));
    cnn_refresh_weights(n->S.N, nullptr);
    VSIE_HIP(hipDeviceSynchronize());
  });
}

int vsie_net_attach(vsie_handle* hd, vsie_net* n) {
  if (!hd) return fail(VSIE_E_ARG, "null handle");
  hd->H.net = n ? &n->S : nullptr;
  if (n) return guarded([&]() { cnn_refresh_weights(n->S.N, hd->H.stream); VSIE_HIP(hipStreamSynchronize(hd->H.stream)); });
  return VSIE_OK;
}

int vsie_net_collect(vsie_net* n, vsie_handle* hd, int nports, const int32_t* ports, const vsie_solve_opts* o,
                     int64_t* n_pairs, void* stream) {
  if (!n || !hd || !ports || nports < 1) return fail(VSIE_E_ARG, "bad argument");
  vsie_solve_opts so;
  int rc = check_solve_opts(hd, o, so);
  if (rc != VSIE_OK) return rc;
  if (so.method != VSIE_SCHUR || !so.precond) return fail(VSIE_E_ARG, "pairs come from the preconditioned SCHUR solve");
  void* x = nullptr;
  rc = guarded([&]() {
    if (hipMalloc(&x, sizeof(cxd) * (size_t)hd->H.N * nports) != hipSuccess) {
      x = nullptr;
      throw Error(VSIE_E_NOMEM, "hipMalloc of the solutions failed");
    }
  });
  if (rc != VSIE_OK) return rc;
  hd->H.collect = &n->S;
  rc = vsie_solve_ports(hd, &so, nports, ports, x, nullptr, stream);
  hd->H.collect = nullptr;
  (void)hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(x);
  if (n_pairs) *n_pairs = n->S.count;
  return rc == VSIE_E_NOCONV ? VSIE_OK : rc;
}

int vsie_net_train(vsie_net* n, int epochs, float lr, uint64_t seed, double* last_loss, void* stream) {
  if (!n || epochs < 1 || !(lr > 0)) return fail(VSIE_E_ARG, "bad argument");
  return guarded([&]() {
    const double l = net_train(n->S, epochs, lr, seed, (hipStream_t)stream);
    if (last_loss) *last_loss = l;
  });
}

__global__ void k_copy_channels(const float* __restrict__ src, int cs, float* __restrict__ dst, int cd, int ncopy,
                                int64_t nvox) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvox * cd; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % cd);
    dst[e] = c < ncopy ? src[(e / cd) * cs + c] : 0.f;
  }
}

int vsie_net_forward(vsie_net* n, int D, int H, int W, const float* x_dev, float* y_dev, void* stream) {
  if (!n || !x_dev || !y_dev) return fail(VSIE_E_ARG, "null argument");
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    Cnn& N = n->S.N;
    cnn_size(N, D, H, W);
    cnn_refresh_weights(N, st);
    const int64_t nvox = (int64_t)D * H * W;
    const unsigned nb = (unsigned)std::min<int64_t>((nvox * 16 + 255) / 256, 65535);
    hipLaunchKernelGGL(k_copy_channels, dim3(nb), dim3(256), 0, st, x_dev, CNN_IN, N.x_in, 16, CNN_IN, nvox);
    cnn_forward(N, st);
    hipLaunchKernelGGL(k_copy_channels, dim3(nb), dim3(256), 0, st, N.act[CNN_NLAYER - 1], 16, y_dev, CNN_OUT, CNN_OUT,
                       nvox);
    VSIE_HIP(hipGetLastError());
  });
}

int vsie_net_gradients(vsie_net* n, int D, int H, int W, const float* x_dev, const float* t_dev, double* loss,
                       float* grads_host, void* stream) {
  if (!n || !x_dev || !t_dev) return fail(VSIE_E_ARG, "null argument");
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    Cnn& N = n->S.N;
    cnn_size(N, D, H, W);
    cnn_refresh_weights(N, st);
    const int64_t nvox = (int64_t)D * H * W;
    const unsigned nb = (unsigned)std::min<int64_t>((nvox * 16 + 255) / 256, 65535);
    hipLaunchKernelGGL(k_copy_channels, dim3(nb), dim3(256), 0, st, x_dev, CNN_IN, N.x_in, 16, CNN_IN, nvox);
    hipLaunchKernelGGL(k_copy_channels, dim3(nb), dim3(256), 0, st, t_dev, CNN_OUT, N.target, 16, CNN_OUT, nvox);
    cnn_forward(N, st);
    cnn_backward(N, st);
    VSIE_HIP(hipGetLastError());
    if (loss) VSIE_HIP(hipMemcpyAsync(loss, N.red, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grads_host) VSIE_HIP(hipMemcpyAsync(grads_host, N.grads, sizeof(float) * N.nparam, hipMemcpyDeviceToHost, st));
    VSIE_HIP(hipStreamSynchronize(st));
  });
}

int vsie_net_adam(vsie_net* n, float lr, void* stream) {
  if (!n || !(lr > 0)) return fail(VSIE_E_ARG, "bad argument");
  return guarded([&]() {
    cnn_adam(n->S.N, lr, (hipStream_t)stream);
    VSIE_HIP(hipGetLastError());
  });
}

int vsie_net_layer(vsie_net* n, int layer, int mode, int D, int H, int W, const float* in0, const float* in1,
                   const float* mask, float* out, void* stream) {
  if (!n || layer < 0 || layer >= CNN_NLAYER || (mode != 0 && mode != 1) || !in0 || !out)
    return fail(VSIE_E_ARG, "bad argument");
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    Cnn& N = n->S.N;
    cnn_refresh_weights(N, st);
    const CnnLayerDesc& d = N.L[layer];
    const bool dec = layer >= 8 && layer <= 10;   // input [up2(a), b], b = the skip
    const int cb = dec ? (layer == 8 ? 48 : layer == 9 ? 32 : 16) : 0;
    if (mode == 0) {
      cnn_conv_forward(st, in0, d.cin_p - cb, dec, dec ? in1 : nullptr, cb, nullptr, N.wf + d.wf_off,
                       N.params + d.b_off, d.relu, out, d.cout_p, d.cout, D, H, W);
    } else {
      cnn_conv_forward(st, in0, d.cout_p, false, nullptr, 0, d.relu ? mask : nullptr, N.wb + d.wb_off, nullptr, false,
                       out, d.cin_p, d.cin_p, D, H, W);
    }
    VSIE_HIP(hipGetLastError());
  });
}

int vsie_net_layer_wgrad(vsie_net* n, int layer, int D, int H, int W, const float* in0, const float* in1,
                         const float* g, const float* mask, float* gw_host, float* gb_host, void* stream) {
  if (!n || layer < 0 || layer >= CNN_NLAYER || !in0 || !g || !gw_host || !gb_host) return fail(VSIE_E_ARG, "bad argument");
  return guarded([&]() {
    hipStream_t st = (hipStream_t)stream;
    Cnn& N = n->S.N;
    const CnnLayerDesc& d = N.L[layer];
    const bool dec = layer >= 8 && layer <= 10;
    const int cb = dec ? (layer == 8 ? 48 : layer == 9 ? 32 : 16) : 0;
    cnn_conv_wgrad(N, st, layer, in0, d.cin_p - cb, dec, dec ? in1 : nullptr, cb, g, d.relu ? mask : nullptr, d.cout_p,
                   N.grads + d.w_off, N.grads + d.b_off, D, H, W);
    VSIE_HIP(hipMemcpyAsync(gw_host, N.grads + d.w_off, sizeof(float) * 27 * d.cout * d.cin, hipMemcpyDeviceToHost, st));
    VSIE_HIP(hipMemcpyAsync(gb_host, N.grads + d.b_off, sizeof(float) * d.cout, hipMemcpyDeviceToHost, st));
    VSIE_HIP(hipStreamSynchronize(st));
  });
}

int vsie_set_concurrency(vsie_handle* hd, int enable) {
  if (!hd) return fail(VSIE_E_ARG, "null handle");
  return guarded([&]() {
    Handle& H = hd->H;
    if (H.side) VSIE_HIP(hipStreamSynchronize(H.side));
    H.concurrent = enable != 0;
  });
}

int vsie_profile(vsie_handle* hd, int enable) { return vsie_profile_mask(hd, enable ? 0xFFFFFFFFu : 0u); }

int vsie_profile_mask(vsie_handle* hd, uint32_t stages) {
  if (!hd) return fail(VSIE_E_ARG, "null handle");
  Handle& H = hd->H;
  const int enable = stages != 0;
  H.prof_stages = stages;
  return guarded([&]() {
    if (enable && !H.ev[0][0])
      for (auto& slot : H.ev)
        for (auto& e : slot) VSIE_HIP(hipEventCreate(&e));
    if (H.prof) drain_profile(H);
    H.ring_count = 0;
    H.prof = enable != 0;
    for (int s = 0; s < Handle::NSTAGE; ++s) {
      H.prof_ms[s] = 0;
      H.prof_calls[s] = 0;
    }
  });
}

int vsie_profile_read(const vsie_handle* hd, int max_stages, const char** names, double* total_ms, int64_t* calls,
                      int* n_stages) {
  if (!hd || !n_stages) return fail(VSIE_E_ARG, "null argument");
  Handle& H = const_cast<vsie_handle*>(hd)->H;   // reading back pending events updates only the totals
  const int rc = guarded([&]() { drain_profile(H); });
  if (rc != VSIE_OK) return rc;
  *n_stages = Handle::NSTAGE;
  for (int s = 0; s < Handle::NSTAGE && s < max_stages; ++s) {
    if (names) names[s] = kStageNames[s];
    if (total_ms) total_ms[s] = H.prof_ms[s];
    if (calls) calls[s] = H.prof_calls[s];
  }
  return VSIE_OK;
}

void vsie_destroy(vsie_handle* hd) { delete hd; }

const char* vsie_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
