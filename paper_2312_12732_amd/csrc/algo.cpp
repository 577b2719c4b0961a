// Algebra of bilinear algorithms <m0,k0,n0;R> on the host: Brent check,
// composition (Kronecker construction, Section 2 of the paper), direct sums,
// re-basis of square algorithms and the built-in coefficient tables.
#include <array>
#include <cmath>
#include <cstring>
#include <string>

#include "mf_internal.h"

namespace mf {

namespace {

bool all_small_integers(const std::vector<double>& x) {
  for (double v : x)
    if (v != std::nearbyint(v) || std::fabs(v) > 1048576.0) return false;
  return true;
}

}  // namespace

int64_t brent_violations(const Algo& a) {
  const int m0 = a.m0, k0 = a.k0, n0 = a.n0, R = a.R;
  const int NA = m0 * k0, NB = k0 * n0, NC = m0 * n0;
  const bool exact = all_small_integers(a.U) && all_small_integers(a.V) && all_small_integers(a.W);
  // Sparse columns of W per product keep the triple loop cheap.
  std::vector<std::vector<std::pair<int, double>>> wcol(R);
  double scale = 1.0;
  for (int r = 0; r < R; ++r)
    for (int c = 0; c < NC; ++c)
      if (a.w(c, r) != 0.0) {
        wcol[r].push_back({c, a.w(c, r)});
        scale = std::fmax(scale, std::fabs(a.w(c, r)));
      }
  int64_t bad = 0;
  std::vector<int64_t> acc_i(NC);
  std::vector<double> acc_d(NC);
  for (int x = 0; x < NA; ++x) {      // A block (i, k)
    for (int y = 0; y < NB; ++y) {    // B block (k2, j)
      std::fill(acc_i.begin(), acc_i.end(), 0);
      std::fill(acc_d.begin(), acc_d.end(), 0.0);
      for (int r = 0; r < R; ++r) {
        const double uv = a.u(x, r) * a.v(y, r);
        if (uv == 0.0) continue;
        for (auto& cw : wcol[r]) {
          if (exact)
            acc_i[cw.first] += (int64_t)uv * (int64_t)cw.second;
          else
            acc_d[cw.first] += uv * cw.second;
        }
      }
      const int i = x / k0, k = x % k0, k2 = y / n0, j = y % n0;
      for (int c = 0; c < NC; ++c) {
        const int want = (k == k2 && c == i * n0 + j) ? 1 : 0;
        if (exact) {
          if (acc_i[c] != want) ++bad;
        } else if (std::fabs(acc_d[c] - want) > 1e-9 * scale * R) {
          ++bad;
        }
      }
    }
  }
  return bad;
}

namespace {

// Kronecker product of two factor matrices X1 (r1 x c1 grid of blocks) and X2
// (r2 x c2 grid): block (I, J) of the (r1 r2) x (c1 c2) grid lies in block
// (I / r2, J / c2) of the outer grid at position (I % r2, J % c2) inside it;
// product r = q1 * R2 + q2 has the product of the two coefficients.
std::vector<double> kron_rows(const std::vector<double>& X1, int r1, int c1, int R1, const std::vector<double>& X2,
                              int r2, int c2, int R2) {
  const int rows = r1 * r2, cols = c1 * c2, R = R1 * R2;
  std::vector<double> out((size_t)rows * cols * R, 0.0);
  for (int I = 0; I < rows; ++I)
    for (int J = 0; J < cols; ++J) {
      const size_t row = (size_t)I * cols + J;
      const int ko = (I / r2) * c1 + (J / c2);
      const int ki = (I % r2) * c2 + (J % c2);
      for (int q1 = 0; q1 < R1; ++q1)
        for (int q2 = 0; q2 < R2; ++q2)
          out[row * R + (size_t)q1 * R2 + q2] = X1[(size_t)ko * R1 + q1] * X2[(size_t)ki * R2 + q2];
    }
  return out;
}

}  // namespace

Algo compose(const Algo& outer, const Algo& inner) {
  Algo c;
  auto flat = [](const Algo& a) {
    if (!a.factors.empty()) return a.factors;
    Algo f = a;
    f.factors.clear();
    return std::vector<Algo>{f};
  };
  c.factors = flat(outer);
  for (const Algo& f : flat(inner)) c.factors.push_back(f);
  const Algo &o = outer, &i = inner;
  c.set_shape(o.m0 * i.m0, o.k0 * i.k0, o.n0 * i.n0);
  c.R = o.R * i.R;
  c.U = kron_rows(o.U, o.m0, o.k0, o.R, i.U, i.m0, i.k0, i.R);
  c.V = kron_rows(o.V, o.k0, o.n0, o.R, i.V, i.k0, i.n0, i.R);
  c.W = kron_rows(o.W, o.m0, o.n0, o.R, i.W, i.m0, i.n0, i.R);
  return c;
}

bool concat(const Algo& a, const Algo& b, int axis, Algo* out) {
  // (rows, cols) of the block grid of each factor matrix of an algorithm
  struct Grid {
    int r, c;
  };
  auto grids = [](const Algo& x) {
    return std::array<Grid, 3>{Grid{x.m0, x.k0}, Grid{x.k0, x.n0}, Grid{x.m0, x.n0}};
  };
  Algo c;
  if (axis == 0 && a.k0 == b.k0 && a.n0 == b.n0)
    c.set_shape(a.m0 + b.m0, a.k0, a.n0);
  else if (axis == 1 && a.m0 == b.m0 && a.n0 == b.n0)
    c.set_shape(a.m0, a.k0 + b.k0, a.n0);
  else if (axis == 2 && a.m0 == b.m0 && a.k0 == b.k0)
    c.set_shape(a.m0, a.k0, a.n0 + b.n0);
  else
    return false;
  c.R = a.R + b.R;
  const auto ga = grids(a), gb = grids(b), gc = grids(c);
  // Which grid dimension of U (A: m, k), V (B: k, n), W (C: m, n) the axis
  // extends: -1 none (both parts use the whole grid), 0 rows, 1 columns.
  const int ext[3][3] = {{0, -1, 0}, {1, 0, -1}, {-1, 1, 1}};  // [axis][matrix]
  std::vector<double>* dst[3] = {&c.U, &c.V, &c.W};
  const std::vector<double>* src_a[3] = {&a.U, &a.V, &a.W};
  const std::vector<double>* src_b[3] = {&b.U, &b.V, &b.W};
  for (int x = 0; x < 3; ++x) {
    dst[x]->assign((size_t)gc[x].r * gc[x].c * c.R, 0.0);
    const int e = ext[axis][x];
    for (int part = 0; part < 2; ++part) {
      const Grid g = part == 0 ? ga[x] : gb[x];
      const std::vector<double>& X = part == 0 ? *src_a[x] : *src_b[x];
      const int R = part == 0 ? a.R : b.R, r0 = part == 0 ? 0 : a.R;
      const int row0 = (part == 1 && e == 0) ? ga[x].r : 0, col0 = (part == 1 && e == 1) ? ga[x].c : 0;
      for (int i = 0; i < g.r; ++i)
        for (int j = 0; j < g.c; ++j)
          for (int q = 0; q < R; ++q)
            (*dst[x])[((size_t)(row0 + i) * gc[x].c + col0 + j) * c.R + r0 + q] = X[((size_t)i * g.c + j) * R + q];
    }
  }
  *out = c;
  return true;
}

Algo power(const Algo& a, int d) {
  Algo out = a;
  for (int i = 1; i < d; ++i) out = compose(out, a);
  return out;
}

namespace {

// Integer inverse of a unimodular p x p matrix; false if none exists.
bool int_inverse(const int64_t* M, int p, std::vector<int64_t>* inv) {
  std::vector<long double> a((size_t)p * 2 * p, 0.0L);
  for (int i = 0; i < p; ++i) {
    for (int j = 0; j < p; ++j) a[(size_t)i * 2 * p + j] = (long double)M[i * p + j];
    a[(size_t)i * 2 * p + p + i] = 1.0L;
  }
  for (int c = 0; c < p; ++c) {
    int piv = c;
    for (int r = c + 1; r < p; ++r)
      if (std::fabs((double)a[(size_t)r * 2 * p + c]) > std::fabs((double)a[(size_t)piv * 2 * p + c])) piv = r;
    if (a[(size_t)piv * 2 * p + c] == 0.0L) return false;
    if (piv != c)
      for (int j = 0; j < 2 * p; ++j) std::swap(a[(size_t)c * 2 * p + j], a[(size_t)piv * 2 * p + j]);
    const long double f = a[(size_t)c * 2 * p + c];
    for (int j = 0; j < 2 * p; ++j) a[(size_t)c * 2 * p + j] /= f;
    for (int r = 0; r < p; ++r) {
      if (r == c) continue;
      const long double g = a[(size_t)r * 2 * p + c];
      if (g == 0.0L) continue;
      for (int j = 0; j < 2 * p; ++j) a[(size_t)r * 2 * p + j] -= g * a[(size_t)c * 2 * p + j];
    }
  }
  inv->assign((size_t)p * p, 0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) (*inv)[i * p + j] = (int64_t)std::llround((double)a[(size_t)i * 2 * p + p + j]);
  // Exact verification M * inv == I.
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      int64_t s = 0;
      for (int k = 0; k < p; ++k) s += M[i * p + k] * (*inv)[k * p + j];
      if (s != (i == j ? 1 : 0)) return false;
    }
  return true;
}

// out = L * X * Rm for p x p matrices (X double, L and Rm integer).
void sandwich(const int64_t* L, bool LT, const double* X, const int64_t* Rm, bool RT, int p, double* out) {
  std::vector<double> tmp((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += (double)(LT ? L[k * p + i] : L[i * p + k]) * X[k * p + j];
      tmp[i * p + j] = s;
    }
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += tmp[i * p + k] * (double)(RT ? Rm[j * p + k] : Rm[k * p + j]);
      out[i * p + j] = s;
    }
}

}  // namespace

bool rebase(const Algo& a, const int64_t* X, const int64_t* Y, const int64_t* Z, Algo* out) {
  if (!a.square()) return false;
  const int p = a.p, P2 = p * p;
  std::vector<int64_t> Xi, Yi, Zi;
  if (!int_inverse(X, p, &Xi) || !int_inverse(Y, p, &Yi) || !int_inverse(Z, p, &Zi)) return false;
  Algo b;
  b.set_shape(p, p, p);
  b.R = a.R;
  b.U.assign((size_t)P2 * a.R, 0.0);
  b.V.assign((size_t)P2 * a.R, 0.0);
  b.W.assign((size_t)P2 * a.R, 0.0);
  std::vector<double> col(P2), res(P2);
  for (int r = 0; r < a.R; ++r) {
    // U'_r = X^T U_r Y^-T
    for (int k = 0; k < P2; ++k) col[k] = a.u(k, r);
    sandwich(X, true, col.data(), Yi.data(), true, p, res.data());
    for (int k = 0; k < P2; ++k) b.U[(size_t)k * a.R + r] = res[k];
    // V'_r = Y^T V_r Z^-T
    for (int k = 0; k < P2; ++k) col[k] = a.v(k, r);
    sandwich(Y, true, col.data(), Zi.data(), true, p, res.data());
    for (int k = 0; k < P2; ++k) b.V[(size_t)k * a.R + r] = res[k];
    // W'_r = X^-1 W_r Z
    for (int k = 0; k < P2; ++k) col[k] = a.w(k, r);
    sandwich(Xi.data(), false, col.data(), Z, false, p, res.data());
    for (int k = 0; k < P2; ++k) b.W[(size_t)k * a.R + r] = res[k];
  }
  *out = b;
  return true;
}

namespace {

Algo from_rows(int p, int R, const int* u, const int* v, const int* w) {
  Algo a;
  a.set_shape(p, p, p);
  a.R = R;
  const int n = p * p * R;
  a.U.assign(u, u + n);
  a.V.assign(v, v + n);
  a.W.assign(w, w + n);
  return a;
}

}  // namespace

// One product A_(i,k) B_(k,j) per (i, j, k), in that loop order, added into
// C_(i,j) (the definition of Section 2, partitioned).
Algo classical_algo(int m0, int k0, int n0) {
  Algo a;
  a.set_shape(m0, k0, n0);
  a.R = m0 * k0 * n0;
  a.U.assign((size_t)m0 * k0 * a.R, 0.0);
  a.V.assign((size_t)k0 * n0 * a.R, 0.0);
  a.W.assign((size_t)m0 * n0 * a.R, 0.0);
  int r = 0;
  for (int i = 0; i < m0; ++i)
    for (int j = 0; j < n0; ++j)
      for (int k = 0; k < k0; ++k, ++r) {
        a.U[(size_t)(i * k0 + k) * a.R + r] = 1.0;
        a.V[(size_t)(k * n0 + j) * a.R + r] = 1.0;
        a.W[(size_t)(i * n0 + j) * a.R + r] = 1.0;
      }
  return a;
}

bool builtin(const std::string& name, Algo* out) {
  if (name == "strassen") {
    // The factor matrices printed in Section 2 (a, b, c^t); the c^t rows are
    // printed for C_0, C_2, C_1, C_3, stored here re-indexed to C_0..C_3.
    static const int u[] = {0, 1, 1, 0, 1, 1, 0,    //
                            0, 0, -1, 1, 0, 0, 0,   //
                            1, 1, 1, 0, 1, 0, 0,    //
                            -1, -1, -1, 0, 0, 0, 1};
    static const int v[] = {0, 0, 0, 0, 1, 1, 0,  //
                            1, 1, 0, 0, 1, 0, 1,  //
                            0, 1, 1, 1, 1, 0, 0,  //
                            0, 1, 1, 0, 1, 0, 1};
    static const int w[] = {0, 0, 0, 1, 0, 1, 0,     // C_0
                            -1, 1, -1, -1, 0, 0, 0,  // C_1 (printed third)
                            0, -1, 0, 0, 1, -1, -1,  // C_2 (printed second)
                            1, 0, 0, 0, 0, 0, 1};    // C_3
    *out = from_rows(2, 7, u, v, w);
    return true;
  }
  if (name == "winograd") {
    // Winograd's form: M0 = A11 B11, M1 = A12 B21, M2 = (A11+A12-A21-A22) B22,
    // M3 = A22 (B11-B12-B21+B22), M4 = (A21+A22)(B12-B11),
    // M5 = (A21+A22-A11)(B11-B12+B22), M6 = (A11-A21)(B22-B12).
    static const int u[] = {1, 0, 1, 0, 0, -1, 1,  //
                            0, 1, 1, 0, 0, 0, 0,   //
                            0, 0, -1, 0, 1, 1, -1, //
                            0, 0, -1, 1, 1, 1, 0};
    static const int v[] = {1, 0, 0, 1, -1, 1, 0,    //
                            0, 0, 0, -1, 1, -1, -1,  //
                            0, 1, 0, -1, 0, 0, 0,    //
                            0, 0, 1, 1, 0, 1, 1};
    static const int w[] = {1, 1, 0, 0, 0, 0, 0,   //
                            1, 0, 1, 0, 1, 1, 0,   //
                            1, 0, 0, -1, 0, 1, 1,  //
                            1, 0, 0, 0, 1, 1, 1};
    *out = from_rows(2, 7, u, v, w);
    return true;
  }
  if (name == "strassen1969") {
    static const int u[] = {1, 0, 1, 0, 1, -1, 0,  //
                            0, 0, 0, 0, 1, 0, 1,   //
                            0, 1, 0, 0, 0, 1, 0,   //
                            1, 1, 0, 1, 0, 0, -1};
    static const int v[] = {1, 1, 0, -1, 0, 1, 0,  //
                            0, 0, 1, 0, 0, 1, 0,   //
                            0, 0, 0, 1, 0, 0, 1,   //
                            1, 0, -1, 0, 1, 0, 1};
    static const int w[] = {1, 0, 0, 1, -1, 0, 1,  //
                            0, 0, 1, 0, 1, 0, 0,   //
                            0, 1, 0, 1, 0, 0, 0,   //
                            1, -1, 1, 0, 0, 1, 0};
    *out = from_rows(2, 7, u, v, w);
    return true;
  }
  if (name == "classical2") {
    *out = classical_algo(2, 2, 2);
    return true;
  }
  if (name == "classical3") {
    *out = classical_algo(3, 3, 3);
    return true;
  }
  return false;
}

}  // namespace mf
