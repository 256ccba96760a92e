// Compile-time structure of the trilinear unit-cube element matrix in the
// element's tensor Haar basis.
//
// For shape functions N_a = phi_ax(x) phi_ay(y) phi_az(z) (phi_0 = 1 - t,
// phi_1 = t) the element matrix of an isotropic material is
//   K_(a,c),(b,e) = lambda G(a,b,c,e) + mu (G(a,b,e,c) + delta_ce sum_d G(a,b,d,d)),
//   G(a,b,c,e)    = integral over the unit cube of dN_a/dx_c dN_b/dx_e.
#pragma once

namespace mgcg {

// The matrix in the element's tensor Haar basis.  With the 1-D modes
// s = (1, 1) and d = (-1, 1) on the element's two nodes along an axis, the
// 3-D mode m = mx + 2 my + 4 mz (mx = 0: s, 1: d) has the node values
// T[a][m] = prod_d h(a_d, m_d), h(0, s) = h(1, s) = h(1, d) = 1, h(0, d) = -1,
// and T T^T = 8 I.  Hence K0 u = T (K_h (T^T u)) with K_h = T^T K0 T / 64:
// the forward transform T^T and the inverse T are sums and differences.
// T^T K0 T is the element's bilinear form on the mode functions, products of
// s(t) = 1 and d(t) = 2t - 1 on [0, 1], whose 1-D integrals are
//   s s: 1, d d: 1/3, s d: 0;  d' s: 2 (d' = 2, s' = 0), d' d: 0;  d' d': 4,
// so K_h is sparse: 45 nonzeros of 576, none in the row or column of the
// constant mode sss (rigid translations).  Scaled by 27 * 64 every lambda-
// and mu-coefficient is an integer, and the nonzeros fall into classes of
// equal (lambda, mu) coefficients up to sign: the kernels keep the class
// values in scalar registers and read class and sign from this table at
// compile time.
struct Q1HaarTable {
  int cls[576];  // -1: structural zero
  int sgn[576];
  int a[16];     // lambda coefficient x 1728 of each class
  int b[16];     // mu coefficient x 1728
  int ncls;
  int nnz;
};

namespace q1detail {

// 3 x the 1-D integral of (mode ma, derivative da) against (mode mb, db).
constexpr int h1d(int ma, int mb, bool da, bool db) {
  if (da && db) return (ma && mb) ? 12 : 0;            // d' d' = 4
  if (da) return (ma && !mb) ? 6 : 0;                  // d' s = 2
  if (db) return (mb && !ma) ? 6 : 0;
  return ma != mb ? 0 : (ma ? 1 : 3);                  // d d = 1/3, s s = 1
}
// 27 x the integral over the unit cube of dN_m/dx_c dN_n/dx_e (mode functions)
constexpr int GH(int m, int n, int c, int e) {
  int p = 1;
  for (int d = 0; d < 3; ++d) p *= h1d((m >> d) & 1, (n >> d) & 1, d == c, d == e);
  return p;
}

constexpr Q1HaarTable build_haar() {
  Q1HaarTable t{};
  t.ncls = 0;
  t.nnz = 0;
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) {
      const int m = i / 3, c = i % 3, n = j / 3, e = j % 3;
      // 27 x (T^T K0 T) = lambda la + mu mb; / 64 for K_h
      int la = GH(m, n, c, e);
      int mb = GH(m, n, e, c);
      if (c == e) mb += GH(m, n, 0, 0) + GH(m, n, 1, 1) + GH(m, n, 2, 2);
      if (la == 0 && mb == 0) {
        t.cls[i * 24 + j] = -1;
        t.sgn[i * 24 + j] = 0;
        continue;
      }
      ++t.nnz;
      const int sg = (la > 0 || (la == 0 && mb > 0)) ? 1 : -1;
      la *= sg;
      mb *= sg;
      int k = -1;
      for (int r = 0; r < t.ncls; ++r)
        if (t.a[r] == la && t.b[r] == mb) k = r;
      if (k < 0) {
        k = t.ncls++;
        t.a[k] = la;
        t.b[k] = mb;
      }
      t.cls[i * 24 + j] = k;
      t.sgn[i * 24 + j] = sg;
    }
  return t;
}

}  // namespace q1detail

constexpr Q1HaarTable kQ1H = q1detail::build_haar();
static_assert(kQ1H.nnz == 45, "trilinear element in the Haar basis: 45 nonzeros expected");
static_assert(kQ1H.ncls <= 16, "Haar class table");
constexpr bool haar_sss_free() {
  for (int q = 0; q < 24; ++q)
    for (int c = 0; c < 3; ++c)
      if (kQ1H.cls[c * 24 + q] >= 0 || kQ1H.cls[q * 24 + c] >= 0) return false;
  return true;
}
static_assert(haar_sss_free(), "the constant mode carries no energy");

template <typename T>
struct Q1HaarVals {
  T v[16];
};

inline Q1HaarVals<double> q1_haar_values(double lambda, double mu) {
  Q1HaarVals<double> out{};
  for (int k = 0; k < kQ1H.ncls; ++k) out.v[k] = (lambda * kQ1H.a[k] + mu * kQ1H.b[k]) / 1728.0;
  return out;
}

}  // namespace mgcg
