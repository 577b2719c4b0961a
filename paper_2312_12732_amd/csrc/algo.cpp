// Algebra of bilinear algorithms <p,p,p;R> on the host: Brent check,
// composition (Kronecker construction, Section 2 of the paper), re-basis and
// the built-in coefficient tables.
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
  const int p = a.p, P2 = p * p, R = a.R;
  const bool exact = all_small_integers(a.U) && all_small_integers(a.V) && all_small_integers(a.W);
  // Sparse columns of W per product keep the triple loop cheap.
  std::vector<std::vector<std::pair<int, double>>> wcol(R);
  double scale = 1.0;
  for (int r = 0; r < R; ++r)
    for (int c = 0; c < P2; ++c)
      if (a.w(c, r) != 0.0) {
        wcol[r].push_back({c, a.w(c, r)});
        scale = std::fmax(scale, std::fabs(a.w(c, r)));
      }
  int64_t bad = 0;
  std::vector<int64_t> acc_i(P2);
  std::vector<double> acc_d(P2);
  for (int x = 0; x < P2; ++x) {      // A block (i, k)
    for (int y = 0; y < P2; ++y) {    // B block (k2, j)
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
      const int i = x / p, k = x % p, k2 = y / p, j = y % p;
      for (int c = 0; c < P2; ++c) {
        const int want = (k == k2 && c == i * p + j) ? 1 : 0;
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

Algo compose(const Algo& outer, const Algo& inner) {
  // Block (I, J) of the fine grid lies in block (I / p2, J / p2) of the outer
  // grid at position (I % p2, J % p2) inside it; product r = r1 * R2 + r2 has
  // the product of the outer and inner coefficients.
  Algo c;
  auto flat = [](const Algo& a) {
    if (!a.factors.empty()) return a.factors;
    Algo f = a;
    f.factors.clear();
    return std::vector<Algo>{f};
  };
  c.factors = flat(outer);
  for (const Algo& f : flat(inner)) c.factors.push_back(f);
  const int p1 = outer.p, p2 = inner.p, R1 = outer.R, R2 = inner.R;
  c.p = p1 * p2;
  c.R = R1 * R2;
  const int P2 = c.p * c.p;
  c.U.assign((size_t)P2 * c.R, 0.0);
  c.V.assign((size_t)P2 * c.R, 0.0);
  c.W.assign((size_t)P2 * c.R, 0.0);
  for (int I = 0; I < c.p; ++I)
    for (int J = 0; J < c.p; ++J) {
      const int row = I * c.p + J;
      const int ko = (I / p2) * p1 + (J / p2);
      const int ki = (I % p2) * p2 + (J % p2);
      for (int r1 = 0; r1 < R1; ++r1)
        for (int r2 = 0; r2 < R2; ++r2) {
          const size_t at = (size_t)row * c.R + (size_t)r1 * R2 + r2;
          c.U[at] = outer.u(ko, r1) * inner.u(ki, r2);
          c.V[at] = outer.v(ko, r1) * inner.v(ki, r2);
          c.W[at] = outer.w(ko, r1) * inner.w(ki, r2);
        }
    }
  return c;
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
  const int p = a.p, P2 = p * p;
  std::vector<int64_t> Xi, Yi, Zi;
  if (!int_inverse(X, p, &Xi) || !int_inverse(Y, p, &Yi) || !int_inverse(Z, p, &Zi)) return false;
  Algo b;
  b.p = p;
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
  a.p = p;
  a.R = R;
  const int n = p * p * R;
  a.U.assign(u, u + n);
  a.V.assign(v, v + n);
  a.W.assign(w, w + n);
  return a;
}

Algo classical(int p) {
  Algo a;
  a.p = p;
  a.R = p * p * p;
  const int P2 = p * p;
  a.U.assign((size_t)P2 * a.R, 0.0);
  a.V.assign((size_t)P2 * a.R, 0.0);
  a.W.assign((size_t)P2 * a.R, 0.0);
  int r = 0;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j)
      for (int k = 0; k < p; ++k, ++r) {
        a.U[(size_t)(i * p + k) * a.R + r] = 1.0;
        a.V[(size_t)(k * p + j) * a.R + r] = 1.0;
        a.W[(size_t)(i * p + j) * a.R + r] = 1.0;
      }
  return a;
}

}  // namespace

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
    *out = classical(2);
    return true;
  }
  if (name == "classical3") {
    *out = classical(3);
    return true;
  }
  return false;
}

}  // namespace mf
