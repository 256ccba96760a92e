// Compile-time structure of the trilinear unit-cube element matrix.
//
// For shape functions N_a = phi_ax(x) phi_ay(y) phi_az(z) (phi_0 = 1 - t,
// phi_1 = t) the element matrix of an isotropic material is
//   K_(a,c),(b,e) = lambda G(a,b,c,e) + mu (G(a,b,e,c) + delta_ce sum_d G(a,b,d,d)),
//   G(a,b,c,e)    = integral over the unit cube of dN_a/dx_c dN_b/dx_e,
// a product of three 1-D integrals (1/3 or 1/6 for phi phi, +-1/2 for a
// derivative against a value, +-1 for two derivatives).  Scaled by 72 every
// lambda- and mu-coefficient is an integer, and the 576 entries fall into 10
// classes of equal (lambda, mu) coefficients up to sign.  The kernels keep the
// 10 class values in scalar registers and read class and sign from this table
// at compile time.
#pragma once

namespace mgcg {

struct Q1Table {
  int cls[576];
  int sgn[576];
  int a72[16];  // lambda coefficient x 72 of each class
  int b72[16];  // mu coefficient x 72 of each class
  int ncls;
};

namespace q1detail {

// 72 x the 1-D integral factor of dimension d.
constexpr int f1d(int ad, int bd, bool da, bool db) {
  const int sa = ad ? 1 : -1, sb = bd ? 1 : -1;
  if (da && db) return 6 * sa * sb;         // 1
  if (da) return 3 * sa;                    // 1/2
  if (db) return 3 * sb;                    // 1/2
  return ad == bd ? 2 : 1;                  // 1/3, 1/6 (x 6)
}

// 72 * G(a, b, c, e) (the per-dimension factors multiply to a multiple of
// 1/72: scale 6 per dimension, divided back by 3 here).
constexpr int G72(int a, int b, int c, int e) {
  int p = 1;
  for (int d = 0; d < 3; ++d) {
    const int ad = (a >> d) & 1, bd = (b >> d) & 1;
    p *= f1d(ad, bd, d == c, d == e);
  }
  return p / 3;  // (6^3 / 72) = 3
}

constexpr Q1Table build() {
  Q1Table t{};
  t.ncls = 0;
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) {
      const int a = i / 3, c = i % 3, b = j / 3, e = j % 3;
      int la = G72(a, b, c, e);
      int mb = G72(a, b, e, c);
      if (c == e) mb += G72(a, b, 0, 0) + G72(a, b, 1, 1) + G72(a, b, 2, 2);
      int s = (la > 0 || (la == 0 && mb > 0)) ? 1 : -1;
      la *= s;
      mb *= s;
      int k = -1;
      for (int q = 0; q < t.ncls; ++q)
        if (t.a72[q] == la && t.b72[q] == mb) k = q;
      if (k < 0) {
        k = t.ncls++;
        t.a72[k] = la;
        t.b72[k] = mb;
      }
      t.cls[i * 24 + j] = k;
      t.sgn[i * 24 + j] = s;
    }
  return t;
}

}  // namespace q1detail

constexpr Q1Table kQ1 = q1detail::build();
static_assert(kQ1.ncls == 10, "trilinear element: 10 coefficient classes expected");

// The 10 class values for Lame constants lambda, mu (unit modulus scaling
// applied by the caller).
template <typename T>
struct Q1Vals {
  T v[10];
};

inline Q1Vals<double> q1_values(double lambda, double mu) {
  Q1Vals<double> out{};
  for (int k = 0; k < 10; ++k) out.v[k] = (lambda * kQ1.a72[k] + mu * kQ1.b72[k]) / 72.0;
  return out;
}

}  // namespace mgcg
