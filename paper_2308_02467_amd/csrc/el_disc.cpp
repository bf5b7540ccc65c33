// Host-side construction of the discretization tables: LGL nodes and weights,
// the nodal differentiation matrix, ordinates, the phase matrix, the
// tau-independent transport blocks B_k - C_k and the local index tables.
//
// Paper references: LGL spectral element (Sec. 2.4.1, eq. sigma_se; the same
// points are the element quadrature points, Fig. 4); local matrices
// (Sec. 2.2.3, eq. hdg_local_all_sub_mat, App. A); Henyey-Greenstein phase
// function (Sec. 2.1); angular partition of the unit circle (Sec. 2.4.1).
#include <cmath>
#include <cstdio>

#include "el_internal.h"

namespace el {

namespace {

// Legendre P_p(x) and P_p'(x) by the three-term recurrences
//   (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1},  P'_{k+1} = P'_{k-1} + (2k+1) P_k.
void legendre(int p, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (p == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 1; k < p; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1;
  *dP = d1;
}

}  // namespace

// Nodes: -1, the p-1 roots of P_p' (Newton from the Chebyshev-Lobatto points,
// second derivative from the Legendre equation), +1.
// Weights: 2 / (p (p+1) P_p(x_i)^2).
bool lgl(int p, double* xi, double* w) {
  if (p < 1 || p > 12) return false;
  xi[0] = -1.0;
  xi[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double x = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, &P, &dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    xi[i] = x;
  }
  for (int i = 0; i <= p; ++i) {
    double P, dP;
    legendre(p, xi[i], &P, &dP);
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
  return true;
}

bool build_disc(const el_disc& d, DiscHost& o, std::string& err) {
  if (d.p < 1 || d.p > 12) { err = "p must be in 1..12"; return false; }
  if (d.n_a < 4 || d.n_a > kMaxNa || d.n_a % 4 != 0) {
    err = "n_a must be a multiple of 4 in 4..64";
    return false;
  }
  if (d.scatter != EL_SCATTER_ISO && d.scatter != EL_SCATTER_HG) { err = "bad scatter kind"; return false; }
  if (d.scatter == EL_SCATTER_HG && !(d.g_hg >= 0.0 && d.g_hg < 1.0)) { err = "g_hg must be in [0,1)"; return false; }
  if (d.angular != EL_ANG_ORDINATES && d.angular != EL_ANG_P0) { err = "bad angular discretization"; return false; }
  o.p = d.p; o.q = d.p + 1; o.n_a = d.n_a; o.nn = o.q * o.q; o.n = o.nn * o.n_a; o.m = 2 * o.q * o.n_a;
  o.scatter = d.scatter; o.g = d.scatter == EL_SCATTER_HG ? d.g_hg : 0.0;
  const int q = o.q, p = o.p, na = o.n_a, nn = o.nn;
  o.xi.assign(q, 0.0); o.omega.assign(q, 0.0);
  lgl(p, o.xi.data(), o.omega.data());
  // D_ij = P_p(x_i) / (P_p(x_j) (x_i - x_j)), D_00 = -p(p+1)/4, D_pp = p(p+1)/4.
  std::vector<double> Pv(q);
  for (int i = 0; i < q; ++i) { double dP; legendre(p, o.xi[i], &Pv[i], &dP); }
  o.D.assign(q * q, 0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      if (i != j) o.D[i * q + j] = Pv[i] / (Pv[j] * (o.xi[i] - o.xi[j]));
  o.D[0] = -p * (p + 1.0) / 4.0;
  o.D[p * q + p] = p * (p + 1.0) / 4.0;
  o.W.assign(nn, 0.0);
  for (int b = 0; b < q; ++b)
    for (int a = 0; a < q; ++a) o.W[b * q + a] = o.omega[a] * o.omega[b];
  // directions of the uniform angular cells: the centre direction
  // (ordinates), or its average over the cell (P0 elements), which is the
  // centre direction times sin(wa/2)/(wa/2)
  const double wa = 2.0 * M_PI / na;
  const double avg = d.angular == EL_ANG_P0 ? std::sin(0.5 * wa) / (0.5 * wa) : 1.0;
  o.sx.resize(na); o.sy.resize(na);
  for (int k = 0; k < na; ++k) {
    double th = (k + 0.5) * wa;
    o.sx[k] = avg * std::cos(th);
    o.sy[k] = avg * std::sin(th);
  }
  // Q[k][k'] = P[k][k'] w_k', rows normalized to sum 1.  The kernel depends
  // on k - k' only: at the centre angle difference (ordinates), or averaged
  // over pairs of cells (P0): the average of p(d wa + x - y) over x, y in
  // [0, wa] is the integral of p(d wa + u) against the triangle
  // (wa - |u|) / wa^2 on [-wa, wa] (Gauss-Legendre on each half).
  const bool hg = o.scatter == EL_SCATTER_HG && o.g != 0.0;
  auto kern = [&](double ang) {
    const double g = o.g;
    return (1.0 - g * g) / std::pow(1.0 + g * g - 2.0 * g * std::cos(ang), 1.5);
  };
  std::vector<double> qd(na, 1.0);
  if (hg) {
    // Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n)
    const int ng = 48;
    std::vector<double> gx(ng), gw(ng);
    for (int i = 0; i < ng; ++i) {
      double x = std::cos(M_PI * (i + 0.75) / (ng + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 1; k < ng; ++k) { double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0); p0 = p1; p1 = p2; }
        const double dp = ng * (x * p1 - p0) / (x * x - 1.0);
        const double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      double p0 = 1.0, p1 = x;
      for (int k = 1; k < ng; ++k) { double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0); p0 = p1; p1 = p2; }
      const double dp = ng * (x * p1 - p0) / (x * x - 1.0);
      gx[i] = x;
      gw[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    for (int dd = 0; dd < na; ++dd) {
      if (d.angular != EL_ANG_P0) { qd[dd] = kern(dd * wa); continue; }
      double acc = 0.0;
      for (int i = 0; i < ng; ++i) {
        const double u = 0.5 * wa * (gx[i] + 1.0);   // [0, wa]
        const double tri = (wa - u) / (wa * wa);
        acc += 0.5 * wa * gw[i] * tri * (kern(dd * wa + u) + kern(dd * wa - u));
      }
      qd[dd] = acc;
    }
  }
  o.Q.assign(na * na, 0.0);
  for (int k = 0; k < na; ++k) {
    double rs = 0.0;
    for (int kp = 0; kp < na; ++kp) {
      const double v = qd[((k - kp) % na + na) % na];
      o.Q[k * na + kp] = v;
      rs += v;
    }
    for (int kp = 0; kp < na; ++kp) o.Q[k * na + kp] /= rs;
  }
  // s_k . n_f
  const double nx[4] = {-1.0, 1.0, 0.0, 0.0}, ny[4] = {0.0, 0.0, -1.0, 1.0};
  auto sn = [&](int k, int f) { return o.sx[k] * nx[f] + o.sy[k] * ny[f]; };
  auto face_node = [&](int f, int j) {
    switch (f) {
      case 0: return j * q;          // W: a = 0, b = j
      case 1: return j * q + p;      // E: a = p, b = j
      case 2: return j;              // S: b = 0, a = j
      default: return p * q + j;     // N: b = p, a = j
    }
  };
  // T_k = B_k - C_k
  o.T.assign((size_t)na * nn * nn, 0.0);
  for (int k = 0; k < na; ++k) {
    double* T = o.T.data() + (size_t)k * nn * nn;
    for (int b = 0; b < q; ++b)
      for (int a = 0; a < q; ++a) {
        int i = b * q + a;
        for (int c = 0; c < q; ++c) T[i * nn + b * q + c] -= o.omega[c] * o.omega[b] * o.sx[k] * o.D[c * q + a];
        for (int dd = 0; dd < q; ++dd) T[i * nn + dd * q + a] -= o.omega[a] * o.omega[dd] * o.sy[k] * o.D[dd * q + b];
      }
    for (int f = 0; f < 4; ++f) {
      double s = sn(k, f);
      if (s > 0)
        for (int j = 0; j < q; ++j) {
          int nd = face_node(f, j);
          T[nd * nn + nd] += o.omega[j] * s;
        }
    }
  }
  // index tables
  o.in_row.clear(); o.out_row.clear(); o.in_val.clear(); o.out_val.clear();
  o.in_f.clear(); o.in_k.clear(); o.in_j.clear(); o.out_f.clear(); o.out_k.clear(); o.out_j.clear();
  for (int f = 0; f < 4; ++f) {
    std::vector<int> If, Of;
    for (int k = 0; k < na; ++k) {
      double s = sn(k, f);
      if (std::fabs(s) < 1e-12) { err = "ordinate tangent to a face"; return false; }
      (s < 0 ? If : Of).push_back(k);
    }
    if ((int)If.size() != na / 2 || (int)Of.size() != na / 2) { err = "non-conforming ordinates"; return false; }
    for (int r = 0; r < na / 2; ++r)
      for (int j = 0; j < q; ++j) {
        int k = If[r], nd = face_node(f, j);
        o.in_row.push_back(k * nn + nd);
        o.in_val.push_back(o.omega[j] * (-sn(k, f)));
        o.in_f.push_back(f); o.in_k.push_back(k); o.in_j.push_back(j);
      }
    for (int r = 0; r < na / 2; ++r)
      for (int j = 0; j < q; ++j) {
        int k = Of[r], nd = face_node(f, j);
        o.out_row.push_back(k * nn + nd);
        o.out_val.push_back(o.omega[j] * sn(k, f));
        o.out_f.push_back(f); o.out_k.push_back(k); o.out_j.push_back(j);
      }
  }
  return true;
}

}  // namespace el
