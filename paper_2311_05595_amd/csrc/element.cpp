// Element stiffness of Lagrange (degree 1-3) and serendipity (degree 2-3)
// hexahedra (Sec. 2 eq. (1), Sec. 2.1; sub-box split of Sec. 3.3), computed
// on the host once per problem.
//
// For an isotropic material with Lame constants lambda, mu the element
// bilinear form, written per pair of shape-function gradients g_a, g_b, is
//   K_(a,c),(b,e) = integral of  lambda g_a[c] g_b[e] + mu g_a[e] g_b[c]
//                              + mu delta_ce (g_a . g_b),
// which equals B^T D B for the Voigt D with engineering shear.  Each
// sub-box of the n^3 split is integrated with (p+1)^3 Gauss-Legendre points
// (exact for these polynomial integrands: the shape functions have degree
// <= p per axis, the serendipity ones included).  Unit element: x = xi / 2.
#include "element.h"

#include <cmath>
#include <stdexcept>

namespace mgcg {

namespace {

// Gauss-Legendre rule on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= m; ++k) {
        double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      double dp = m * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= m; ++k) {
      double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    double dp = m * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// 1-D Lagrange basis of degree p on equally spaced nodes of [-1, 1]:
// values l[k] and derivatives d[k] at t.
void basis_1d(int p, double t, double* l, double* d) {
  double nodes[4];
  for (int k = 0; k <= p; ++k) nodes[k] = -1.0 + 2.0 * k / p;
  for (int k = 0; k <= p; ++k) {
    double v = 1.0, dv = 0.0;
    for (int m = 0; m <= p; ++m) {
      if (m == k) continue;
      double f = 1.0 / (nodes[k] - nodes[m]);
      // product rule, accumulated incrementally
      dv = dv * (t - nodes[m]) * f + v * f;
      v = v * (t - nodes[m]) * f;
    }
    l[k] = v;
    d[k] = dv;
  }
}

// Local gradients of the 20-node serendipity shape functions at (t0, t1, t2),
// written into the 27-node layout (zero at face and body centres).  Node a
// has local coordinates c_d = a_d - 1 in {-1, 0, 1}.  A vertex function is
// (1 + c0 t0)(1 + c1 t1)(1 + c2 t2)(c0 t0 + c1 t1 + c2 t2 - 2) / 8; an edge
// midpoint with c_m = 0 has (1 - t_m^2) times the two linear factors, / 4.
void serendipity_grad(const double t[3], double* grad) {
  for (int a = 0; a < 27; ++a) {
    const int c[3] = {a % 3 - 1, (a / 3) % 3 - 1, a / 9 - 1};
    const int zeros = (c[0] == 0) + (c[1] == 0) + (c[2] == 0);
    double* g = &grad[3 * a];
    g[0] = g[1] = g[2] = 0.0;
    if (zeros == 0) {
      double f[3];
      for (int d = 0; d < 3; ++d) f[d] = 1.0 + c[d] * t[d];
      const double s = c[0] * t[0] + c[1] * t[1] + c[2] * t[2] - 2.0;
      for (int d = 0; d < 3; ++d) {
        const double others = f[(d + 1) % 3] * f[(d + 2) % 3];
        g[d] = 0.125 * c[d] * others * (s + f[d]);
      }
    } else if (zeros == 1) {
      double f[3], df[3];
      for (int d = 0; d < 3; ++d) {
        if (c[d] == 0) {
          f[d] = 1.0 - t[d] * t[d];
          df[d] = -2.0 * t[d];
        } else {
          f[d] = 1.0 + c[d] * t[d];
          df[d] = c[d];
        }
      }
      g[0] = 0.25 * df[0] * f[1] * f[2];
      g[1] = 0.25 * f[0] * df[1] * f[2];
      g[2] = 0.25 * f[0] * f[1] * df[2];
    }
  }
}

// Local gradients of the 32-node cubic serendipity shape functions at
// (t0, t1, t2), in the 64-node layout (zero at face- and body-interior
// nodes).  Node a has local coordinates c_d = -1 + 2 a_d / 3.  A vertex
// function is (1 + c0 t0)(1 + c1 t1)(1 + c2 t2)(9 |t|^2 - 19) / 64; an edge
// node with |c_m| = 1/3 has 9 (1 - t_m^2)(1 + 9 c_m t_m) times the two
// linear factors, / 64.
void serendipity3_grad(const double t[3], double* grad) {
  for (int a = 0; a < 64; ++a) {
    const int q[3] = {a % 4, (a / 4) % 4, a / 16};
    double c[3];
    int inner = 0, m = -1;
    for (int d = 0; d < 3; ++d) {
      c[d] = -1.0 + 2.0 * q[d] / 3.0;
      if (q[d] == 1 || q[d] == 2) {
        ++inner;
        m = d;
      }
    }
    double* g = &grad[3 * a];
    g[0] = g[1] = g[2] = 0.0;
    if (inner == 0) {
      double f[3];
      for (int d = 0; d < 3; ++d) f[d] = 1.0 + c[d] * t[d];
      const double s = 9.0 * (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) - 19.0;
      for (int d = 0; d < 3; ++d)
        g[d] = f[(d + 1) % 3] * f[(d + 2) % 3] * (c[d] * s + 18.0 * t[d] * f[d]) / 64.0;
    } else if (inner == 1) {
      double f[3], df[3];
      for (int d = 0; d < 3; ++d) {
        if (d == m) {
          f[d] = (1.0 - t[d] * t[d]) * (1.0 + 9.0 * c[d] * t[d]);
          df[d] = -2.0 * t[d] * (1.0 + 9.0 * c[d] * t[d]) + 9.0 * c[d] * (1.0 - t[d] * t[d]);
        } else {
          f[d] = 1.0 + c[d] * t[d];
          df[d] = c[d];
        }
      }
      g[0] = 9.0 * df[0] * f[1] * f[2] / 64.0;
      g[1] = 9.0 * f[0] * df[1] * f[2] / 64.0;
      g[2] = 9.0 * f[0] * f[1] * df[2] / 64.0;
    }
  }
}

}  // namespace

std::vector<double> sub_element_matrices(int order, int nsub, double nu, int family) {
  if (order < 1 || order > 3 || nsub < 1) throw std::invalid_argument("element order/nsub");
  if (family != 0 && !(family == 1 && order >= 2))
    throw std::invalid_argument("serendipity elements have degree 2 or 3");
  const int p1 = order + 1;
  const int nen = p1 * p1 * p1;
  const int nd = 3 * nen;
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double dxi_dx = 2.0;       // unit element: x = xi / 2
  const double jac = 0.125;        // dx dy dz = (1/8) dxi deta dzeta
  std::vector<double> gx, gw;
  gauss_legendre(p1, gx, gw);

  const int ns3 = nsub * nsub * nsub;
  std::vector<double> out((size_t)ns3 * nd * nd, 0.0);
  std::vector<double> grad((size_t)nen * 3);
  for (int sz = 0; sz < nsub; ++sz)
    for (int sy = 0; sy < nsub; ++sy)
      for (int sx = 0; sx < nsub; ++sx) {
        double* K = &out[(size_t)(sx + nsub * (sy + nsub * sz)) * nd * nd];
        const int s[3] = {sx, sy, sz};
        double lo[3], half[3];
        for (int d = 0; d < 3; ++d) {
          lo[d] = -1.0 + 2.0 * s[d] / nsub;
          half[d] = 1.0 / nsub;  // half-length of the sub-interval (length 2/n)
        }
        for (int qz = 0; qz < p1; ++qz)
          for (int qy = 0; qy < p1; ++qy)
            for (int qx = 0; qx < p1; ++qx) {
              const int q[3] = {qx, qy, qz};
              double L[3][4], D[3][4], tq[3];
              double wq = jac;
              for (int d = 0; d < 3; ++d) {
                double t = lo[d] + half[d] * (gx[q[d]] + 1.0);
                tq[d] = t;
                basis_1d(order, t, L[d], D[d]);
                wq *= gw[q[d]] * half[d];
              }
              if (family == 1) {
                if (order == 2)
                  serendipity_grad(tq, grad.data());
                else
                  serendipity3_grad(tq, grad.data());
                for (double& v : grad) v *= dxi_dx;
              } else {
                for (int az = 0; az < p1; ++az)
                  for (int ay = 0; ay < p1; ++ay)
                    for (int ax = 0; ax < p1; ++ax) {
                      int a = ax + p1 * (ay + p1 * az);
                      grad[3 * a + 0] = dxi_dx * D[0][ax] * L[1][ay] * L[2][az];
                      grad[3 * a + 1] = dxi_dx * L[0][ax] * D[1][ay] * L[2][az];
                      grad[3 * a + 2] = dxi_dx * L[0][ax] * L[1][ay] * D[2][az];
                    }
              }
              for (int a = 0; a < nen; ++a)
                for (int b = 0; b < nen; ++b) {
                  const double* ga = &grad[3 * a];
                  const double* gb = &grad[3 * b];
                  double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
                  for (int c = 0; c < 3; ++c)
                    for (int e = 0; e < 3; ++e) {
                      double v = lam * ga[c] * gb[e] + mu * ga[e] * gb[c];
                      if (c == e) v += mu * dot;
                      K[(size_t)(3 * a + c) * nd + 3 * b + e] += wq * v;
                    }
                }
            }
      }
  return out;
}

double trilinear_weight(int px, int py, int pz, int b, int r) {
  auto w1 = [r](int pos, int bit) -> double {
    return bit ? (double)pos / r : (double)(r - pos) / r;
  };
  return w1(px, b & 1) * w1(py, (b >> 1) & 1) * w1(pz, (b >> 2) & 1);
}

}  // namespace mgcg
