// Scalar and complex arithmetic, Green functions and quadrature primitives shared by the
// device setup kernels and the host-side setup code of the library.
//
// Conventions: time dependence exp(+i w t); g(R) = exp(-i k R) / (4 pi R); every row of the
// coupled system multiplied by i w eps0; PWC voxel currents; RWG surface currents.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#define VHD __host__ __device__ inline

namespace vsie {

template <typename R> struct cx {
  R re, im;
};
using cxd = cx<double>;
using cxf = cx<float>;

template <typename R> VHD cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> VHD cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> VHD cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> VHD cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> VHD cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> VHD cx<R>& operator+=(cx<R>& a, cx<R> b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
template <typename R> VHD cx<R>& operator-=(cx<R>& a, cx<R> b) {
  a.re -= b.re;
  a.im -= b.im;
  return a;
}
template <typename R> VHD cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// a * b^* and a^* * b
template <typename R> VHD cx<R> mul_conj_b(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R> VHD cx<R> mul_conj_a(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
VHD cxd cinv(cxd a) {
  double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}

constexpr double PI = 3.14159265358979323846;
constexpr double EPS0 = 8.8541878128e-12;
constexpr double MU0 = 1.25663706212e-6;

// ---------------------------------------------------------------------------------------------
// Gauss-Legendre tables on [0, 1] for n = 1 .. GMAX points, computed once on the host by Newton
// iteration on the Legendre three-term recurrence (no external library).
constexpr int GMAX = 20;
struct GaussTab {
  double x[GMAX + 1][GMAX];
  double w[GMAX + 1][GMAX];
};
void fill_gauss_table(GaussTab* t);  // host

// ---------------------------------------------------------------------------------------------
// Voxel-pair integrals. All lengths in units of the voxel edge h; kappa = k0 h;
// K(rho) = exp(-i kappa rho) / (4 pi rho).
//
// cell integral over the unit cell [lo, lo+1]^D of K(sqrt(|x - c|^2 + delta^2)) * prod w_i(x_i),
// w_i = 1 - |x_i| on axes flagged in `tent`, 1 otherwise. A cell touched by the point (c, delta)
// must have c at a corner; it is integrated after the Duffy map (pyramids in 3D, triangles in
// 2D) with a fixed Gauss order. Other cells lie at least one cell away and use a tensor Gauss
// rule whose order follows from the Bernstein-ellipse bound at that distance.
struct CellRule {
  int n_duffy;     // Gauss points per direction inside Duffy-mapped cells
  double digits;   // target digits for the regular cells
  int n_min, n_max;
};

VHD int regular_order(double dist, const CellRule& cr) {
  // z = -1 + 2 i dist in the cell's [-1,1] coordinate; rho = |z + sqrt(z^2 - 1)| (outer branch)
  double zr = -1.0, zi = 2.0 * dist;
  // z^2 - 1
  double ar = zr * zr - zi * zi - 1.0, ai = 2.0 * zr * zi;
  double mod = sqrt(sqrt(ar * ar + ai * ai));
  double ang = 0.5 * atan2(ai, ar);
  double sr = mod * cos(ang), si = mod * sin(ang);
  double r1 = sqrt((zr + sr) * (zr + sr) + (zi + si) * (zi + si));
  double r2 = sqrt((zr - sr) * (zr - sr) + (zi - si) * (zi - si));
  double rho = r1 > r2 ? r1 : r2;
  int n = (int)ceil(cr.digits * 2.302585092994046 / (2.0 * log(rho)));
  if (n < cr.n_min) n = cr.n_min;
  if (n > cr.n_max) n = cr.n_max;
  return n;
}

VHD cxd kernel_K(double r, double kappa) {
  double s, c;
  sincos(kappa * r, &s, &c);
  double f = 1.0 / (4.0 * PI * r);
  return {c * f, -s * f};
}

template <int D>
VHD cxd cell_integral(const GaussTab& gt, const double* lo, const double* c, double delta,
                      const bool* tent, double kappa, const CellRule& cr) {
  double gap2 = 0.0;
  for (int i = 0; i < D; ++i) {
    double g = lo[i] - c[i];
    double g2 = c[i] - lo[i] - 1.0;
    if (g2 > g) g = g2;
    if (g < 0.0) g = 0.0;
    gap2 += g * g;
  }
  double dist = sqrt(gap2 + delta * delta);
  cxd acc = {0.0, 0.0};
  if (dist == 0.0) {
    double sg[D];
    for (int i = 0; i < D; ++i) sg[i] = (c[i] == lo[i]) ? 1.0 : -1.0;
    const int n = cr.n_duffy;
    const double* X = gt.x[n];
    const double* Wt = gt.w[n];
    if (D == 3) {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
          for (int e = 0; e < n; ++e) {
            double t = X[a], u = X[b], v = X[e];
            double wgt = Wt[a] * Wt[b] * Wt[e];
            double s = sqrt(1.0 + u * u + v * v);
            double rr = t * s;
            double sn, cs;
            sincos(kappa * rr, &sn, &cs);
            // K(r) t^2 = exp(-i kappa r) t / (4 pi s)
            double base = wgt * t / (4.0 * PI * s);
            for (int j = 0; j < 3; ++j) {
              double y[3];
              y[j] = t;
              y[(j + 1) % 3] = t * u;
              y[(j + 2) % 3] = t * v;
              double w = 1.0;
              for (int i = 0; i < 3; ++i)
                if (tent[i]) w *= 1.0 - fabs(c[i] + sg[i] * y[i]);
              acc.re += base * w * cs;
              acc.im -= base * w * sn;
            }
          }
    } else {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          double t = X[a], u = X[b];
          double wgt = Wt[a] * Wt[b];
          double s = sqrt(1.0 + u * u);
          double rr = t * s;
          double sn, cs;
          sincos(kappa * rr, &sn, &cs);
          double base = wgt / (4.0 * PI * s);   // K(r) t = exp(-i kappa r) / (4 pi s)
          for (int j = 0; j < 2; ++j) {
            double y[2];
            y[j] = t;
            y[1 - j] = t * u;
            double w = 1.0;
            for (int i = 0; i < 2; ++i)
              if (tent[i]) w *= 1.0 - fabs(c[i] + sg[i] * y[i]);
            acc.re += base * w * cs;
            acc.im -= base * w * sn;
          }
        }
    }
    return acc;
  }
  const int n = regular_order(dist, cr);
  const double* X = gt.x[n];
  const double* Wt = gt.w[n];
  if (D == 3) {
    for (int a = 0; a < n; ++a) {
      double x0 = lo[0] + X[a];
      double d0 = x0 - c[0];
      double w0 = Wt[a] * (tent[0] ? 1.0 - fabs(x0) : 1.0);
      for (int b = 0; b < n; ++b) {
        double x1 = lo[1] + X[b];
        double d1 = x1 - c[1];
        double w1 = w0 * Wt[b] * (tent[1] ? 1.0 - fabs(x1) : 1.0);
        for (int e = 0; e < n; ++e) {
          double x2 = lo[2] + X[e];
          double d2 = x2 - c[2];
          double w2 = w1 * Wt[e] * (tent[2] ? 1.0 - fabs(x2) : 1.0);
          double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2 + delta * delta);
          cxd k = kernel_K(r, kappa);
          acc.re += w2 * k.re;
          acc.im += w2 * k.im;
        }
      }
    }
  } else {
    for (int a = 0; a < n; ++a) {
      double x0 = lo[0] + X[a];
      double d0 = x0 - c[0];
      double w0 = Wt[a] * (tent[0] ? 1.0 - fabs(x0) : 1.0);
      for (int b = 0; b < n; ++b) {
        double x1 = lo[1] + X[b];
        double d1 = x1 - c[1];
        double w1 = w0 * Wt[b] * (tent[1] ? 1.0 - fabs(x1) : 1.0);
        double r = sqrt(d0 * d0 + d1 * d1 + delta * delta);
        cxd k = kernel_K(r, kappa);
        acc.re += w1 * k.re;
        acc.im += w1 * k.im;
      }
    }
  }
  return acc;
}

// V(d) = int_{[-1,1]^3} K(|t + d|) prod(1 - |t_i|) dt
VHD cxd vol_V(const GaussTab& gt, double d0, double d1, double d2, double kappa, const CellRule& cr) {
  const bool tent[3] = {true, true, true};
  const double c[3] = {-d0, -d1, -d2};
  cxd acc = {0, 0};
  for (int cz = -1; cz <= 0; ++cz)
    for (int cy = -1; cy <= 0; ++cy)
      for (int cxx = -1; cxx <= 0; ++cxx) {
        const double lo[3] = {(double)cxx, (double)cy, (double)cz};
        acc += cell_integral<3>(gt, lo, c, 0.0, tent, kappa, cr);
      }
  return acc;
}

// F2(s; e) = int_{[-1,1]^2} K(sqrt(s^2 + |t + e|^2)) prod(1 - |t_i|) dt
VHD cxd face_F2(const GaussTab& gt, double s, double e0, double e1, double kappa, const CellRule& cr) {
  const bool tent[2] = {true, true};
  const double c[2] = {-e0, -e1};
  cxd acc = {0, 0};
  for (int cy = -1; cy <= 0; ++cy)
    for (int cxx = -1; cxx <= 0; ++cxx) {
      const double lo[2] = {(double)cxx, (double)cy};
      acc += cell_integral<2>(gt, lo, c, fabs(s), tent, kappa, cr);
    }
  return acc;
}

// G(m, n; dc) = int_m^{m+1} dX int_n^{n+1} dY int_{-1}^{1} (1 - |t|) K(|(X, Y, t - dc)|) dt
VHD cxd face_G(const GaussTab& gt, double m, double n, double dc, double kappa, const CellRule& cr) {
  const bool tent[3] = {false, false, true};
  const double c[3] = {0.0, 0.0, dc};
  cxd acc = {0, 0};
  for (int ct = -1; ct <= 0; ++ct) {
    const double lo[3] = {m, n, (double)ct};
    acc += cell_integral<3>(gt, lo, c, 0.0, tent, kappa, cr);
  }
  return acc;
}

// Dimensionless Toeplitz generator at integer offset d (six components xx yy zz xy xz yz):
//   T_aa = -kappa^2 V(d) + 2 F2(d_a) - F2(d_a - 1) - F2(d_a + 1)
//   T_ab = -[G(d_a, d_b) - G(d_a - 1, d_b) - G(d_a, d_b - 1) + G(d_a - 1, d_b - 1)]   (c = third axis)
VHD void generator_T(const GaussTab& gt, int d0, int d1, int d2, double kappa, const CellRule& cr,
                     cxd out[6]) {
  const double d[3] = {(double)d0, (double)d1, (double)d2};
  cxd V = vol_V(gt, d[0], d[1], d[2], kappa, cr);
  for (int a = 0; a < 3; ++a) {
    double e0 = d[(a + 1) % 3], e1 = d[(a + 2) % 3];
    cxd f0 = face_F2(gt, d[a], e0, e1, kappa, cr);
    cxd fm = face_F2(gt, d[a] - 1.0, e0, e1, kappa, cr);
    cxd fp = face_F2(gt, d[a] + 1.0, e0, e1, kappa, cr);
    cxd t = 2.0 * f0 - fm - fp;
    t.re -= kappa * kappa * V.re;
    t.im -= kappa * kappa * V.im;
    out[a] = t;
  }
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int q = 0; q < 3; ++q) {
    int a = pa[q], b = pb[q], c = 3 - a - b;
    if (d[a] == 0.0 || d[b] == 0.0) {
      out[3 + q] = {0.0, 0.0};
      continue;
    }
    cxd g00 = face_G(gt, d[a], d[b], d[c], kappa, cr);
    cxd g10 = face_G(gt, d[a] - 1.0, d[b], d[c], kappa, cr);
    cxd g01 = face_G(gt, d[a], d[b] - 1.0, d[c], kappa, cr);
    cxd g11 = face_G(gt, d[a] - 1.0, d[b] - 1.0, d[c], kappa, cr);
    cxd t = g00 - g10 - g01 + g11;
    out[3 + q] = {-t.re, -t.im};
  }
}

// ---------------------------------------------------------------------------------------------
// Surface rules. R5: 5-point triangle rule, exact to total degree 3, positive weights; the
// "5 surface points" of the coupling integrals. Barycentric coordinates and area fractions.
struct TriRule5 {
  static constexpr int N = 5;
};
VHD void r5_point(int q, double* l, double* w) {
  const double L[5][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
                          {0.66, 0.17, 0.17},
                          {0.082832331329325317301, 0.45858383433533734135, 0.45858383433533734135},
                          {0.2, 0.70704891655600176715, 0.092951083443998232846},
                          {0.2, 0.092951083443998232846, 0.70704891655600176715}};
  const double W[5] = {0.03, 0.33127923434407885754, 0.19677027567856090582, 0.22097524498868011832,
                       0.22097524498868011832};
  l[0] = L[q][0];
  l[1] = L[q][1];
  l[2] = L[q][2];
  *w = W[q];
}

struct V3 {
  double x, y, z;
};
VHD V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
VHD V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
VHD V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
VHD double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
VHD V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
VHD double norm(V3 a) { return sqrt(dot(a, a)); }

// Closed-form static integrals over a flat triangle q0 q1 q2 for the point r:
//   s0 = int_T 1/R dS',  s1 = int_T (r' - r)/R dS'
VHD void triangle_static(V3 r, V3 q0, V3 q1, V3 q2, double* s0, V3* s1) {
  V3 n = cross(q1 - q0, q2 - q0);
  n = (1.0 / norm(n)) * n;
  double d = dot(r - q0, n);
  double ad = fabs(d);
  V3 rho = r - d * n;
  const V3 Q[3] = {q0, q1, q2};
  double S0 = 0.0;
  V3 SV = {0, 0, 0};
  for (int e = 0; e < 3; ++e) {
    V3 qa = Q[e], qb = Q[(e + 1) % 3];
    V3 L = qb - qa;
    V3 sh = (1.0 / norm(L)) * L;
    V3 mh = cross(sh, n);
    double sm = dot(qa - rho, sh);
    double sp = dot(qb - rho, sh);
    double t0 = dot(qa - rho, mh);
    double Rm = norm(r - qa);
    double Rp = norm(r - qb);
    double R02 = t0 * t0 + d * d;
    double lg = 0.0;
    if (R02 > 0.0) {
      double num = (sp >= 0.0) ? log(Rp + sp) : log(R02) - log(Rp - sp);
      double den = (sm >= 0.0) ? log(Rm + sm) : log(R02) - log(Rm - sm);
      lg = num - den;
    }
    double at = 0.0;
    if (ad > 0.0) at = atan(t0 * sp / (R02 + ad * Rp)) - atan(t0 * sm / (R02 + ad * Rm));
    if (t0 != 0.0) S0 += t0 * lg;
    S0 -= ad * at;
    SV = SV + (0.5 * (R02 * lg + sp * Rp - sm * Rm)) * mh;
  }
  *s0 = S0;
  *s1 = SV - (d * S0) * n;
}

// (exp(-i k R) - 1) / R with the limit -i k at R = 0
VHD cxd phi_dyn(double R, double k) {
  if (R <= 0.0) return {0.0, -k};
  double s = sin(0.5 * k * R);
  return {-2.0 * s * s / R, -sin(k * R) / R};
}

VHD cxd green(double R, double k) {
  double s, c;
  sincos(k * R, &s, &c);
  double f = 1.0 / (4.0 * PI * R);
  return {c * f, -s * f};
}

// Triangle-pair moments of the EFIE for testing triangle A (outer R5 rule) and source triangle
// B (closed-form static part + R5 on exp(-ikR)-1 over R):
//   Bm = int_A int_B g,   Am[a][b] = int_A int_B (r - va_a).(r' - vb_b) g
VHD void tri_pair_oriented(const V3* va, const V3* vb, double areaA, double areaB, double k, cxd* Bm,
                           cxd Am[3][3]) {
  double wq[5];
  V3 ra[5], rb[5];
  for (int q = 0; q < 5; ++q) {
    double l[3], w;
    r5_point(q, l, &w);
    wq[q] = w;
    ra[q] = l[0] * va[0] + l[1] * va[1] + l[2] * va[2];
    rb[q] = l[0] * vb[0] + l[1] * vb[1] + l[2] * vb[2];
  }
  cxd sumI = {0, 0};          // sum wq I0
  cxd sum_rM = {0, 0};        // sum wq r.M
  cxd tIr[3] = {{0, 0}, {0, 0}, {0, 0}};   // sum wq I0 r
  cxd tM[3] = {{0, 0}, {0, 0}, {0, 0}};    // sum wq M
  const double inv4pi = 1.0 / (4.0 * PI);
  for (int q = 0; q < 5; ++q) {
    double s0;
    V3 s1;
    triangle_static(ra[q], vb[0], vb[1], vb[2], &s0, &s1);
    cxd ph = {0, 0};
    cxd pr[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int j = 0; j < 5; ++j) {
      double R = norm(ra[q] - rb[j]);
      cxd p = (wq[j] * areaB) * phi_dyn(R, k);
      ph += p;
      pr[0] += rb[j].x * p;
      pr[1] += rb[j].y * p;
      pr[2] += rb[j].z * p;
    }
    cxd I0 = {(s0 + ph.re) * inv4pi, ph.im * inv4pi};
    cxd M[3] = {{(ra[q].x * s0 + s1.x + pr[0].re) * inv4pi, pr[0].im * inv4pi},
                {(ra[q].y * s0 + s1.y + pr[1].re) * inv4pi, pr[1].im * inv4pi},
                {(ra[q].z * s0 + s1.z + pr[2].re) * inv4pi, pr[2].im * inv4pi}};
    double w = wq[q] * areaA;
    sumI += w * I0;
    cxd rM = ra[q].x * M[0] + ra[q].y * M[1] + ra[q].z * M[2];
    sum_rM += w * rM;
    tIr[0] += (w * ra[q].x) * I0;
    tIr[1] += (w * ra[q].y) * I0;
    tIr[2] += (w * ra[q].z) * I0;
    tM[0] += w * M[0];
    tM[1] += w * M[1];
    tM[2] += w * M[2];
  }
  *Bm = sumI;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cxd v = sum_rM;
      v -= vb[b].x * tIr[0] + vb[b].y * tIr[1] + vb[b].z * tIr[2];
      v -= va[a].x * tM[0] + va[a].y * tM[1] + va[a].z * tM[2];
      v += dot(va[a], vb[b]) * sumI;
      Am[a][b] = v;
    }
}

// Pure R5 x R5 rule (used for well-separated triangle pairs; symmetric by construction)
VHD void tri_pair_r5r5(const V3* va, const V3* vb, double areaA, double areaB, double k, cxd* Bm,
                       cxd Am[3][3]) {
  double wq[5];
  V3 ra[5], rb[5];
  for (int q = 0; q < 5; ++q) {
    double l[3], w;
    r5_point(q, l, &w);
    wq[q] = w;
    ra[q] = l[0] * va[0] + l[1] * va[1] + l[2] * va[2];
    rb[q] = l[0] * vb[0] + l[1] * vb[1] + l[2] * vb[2];
  }
  cxd B = {0, 0};
  cxd Ar[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Ar[a][b] = {0, 0};
  for (int q = 0; q < 5; ++q)
    for (int j = 0; j < 5; ++j) {
      double R = norm(ra[q] - rb[j]);
      cxd gv = (wq[q] * areaA * wq[j] * areaB) * green(R, k);
      B += gv;
      for (int a = 0; a < 3; ++a) {
        V3 pa = ra[q] - va[a];
        for (int b = 0; b < 3; ++b) Ar[a][b] += dot(pa, rb[j] - vb[b]) * gv;
      }
    }
  *Bm = B;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Am[a][b] = Ar[a][b];
}

// Classification of a triangle pair: "near" when the squared centroid distance is below
// (4 * longest edge of the pair)^2. Computed with explicit rounded operations so that the
// decision does not depend on contraction into fused multiply-adds.
VHD double sq_rn(V3 a) {
#ifdef __HIP_DEVICE_COMPILE__
  return __dadd_rn(__dadd_rn(__dmul_rn(a.x, a.x), __dmul_rn(a.y, a.y)), __dmul_rn(a.z, a.z));
#else
  volatile double x = a.x * a.x;
  volatile double y = a.y * a.y;
  volatile double z = a.z * a.z;
  volatile double s = x + y;
  return s + z;
#endif
}

VHD bool tri_pair_near(const V3* va, const V3* vb) {
  V3 ca = (1.0 / 3.0) * (va[0] + va[1] + va[2]);
  V3 cb = (1.0 / 3.0) * (vb[0] + vb[1] + vb[2]);
  double d2 = sq_rn(ca - cb);
  double e2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    double ea = sq_rn(va[(i + 1) % 3] - va[i]);
    double eb = sq_rn(vb[(i + 1) % 3] - vb[i]);
    if (ea > e2) e2 = ea;
    if (eb > e2) e2 = eb;
  }
  return d2 < 16.0 * e2;
}

// Symmetric triangle-pair moments (average of both orderings for near pairs)
VHD void tri_pair_moments(const V3* va, const V3* vb, double areaA, double areaB, double k, cxd* Bm,
                          cxd Am[3][3]) {
  if (!tri_pair_near(va, vb)) {
    tri_pair_r5r5(va, vb, areaA, areaB, k, Bm, Am);
    return;
  }
  cxd B1, B2, A1[3][3], A2[3][3];
  tri_pair_oriented(va, vb, areaA, areaB, k, &B1, A1);
  tri_pair_oriented(vb, va, areaB, areaA, k, &B2, A2);
  *Bm = 0.5 * (B1 + B2);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Am[a][b] = 0.5 * (A1[a][b] + A2[b][a]);
}

// (k^2 I + grad grad) g (R) applied to v
VHD void dyad_apply(V3 R, const cxd v[3], double k, cxd out[3]) {
  double r = norm(R);
  cxd g = green(r, k);
  cxd a = {k * k - 1.0 / (r * r), -k / r};
  cxd b = {3.0 / (r * r) - k * k, 3.0 * k / r};
  cxd rv = (R.x / (r * r)) * v[0] + (R.y / (r * r)) * v[1] + (R.z / (r * r)) * v[2];
  cxd brv = b * rv;
  const double Rc[3] = {R.x, R.y, R.z};
  for (int i = 0; i < 3; ++i) out[i] = g * (a * v[i] + Rc[i] * brv);
}

}  // namespace vsie
