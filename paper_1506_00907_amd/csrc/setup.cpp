// Host-side set-up (FP64): reference element, connectivity, geometry, multi-rate levels.
// Compiled with -ffp-contract=off so that the level assignment is reproducible.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace dgrtm {

// ---------------------------------------------------------------------------------------------
// orthonormal Jacobi polynomials P_n^(alpha,beta) on [-1,1] (three-term recurrence)
// ---------------------------------------------------------------------------------------------
static double jacobi(double x, double al, double be, int n) {
  double g0 = std::pow(2.0, al + be + 1.0) / (al + be + 1.0) * std::tgamma(al + 1.0) * std::tgamma(be + 1.0) /
              std::tgamma(al + be + 1.0);
  double p0 = 1.0 / std::sqrt(g0);
  if (n == 0) return p0;
  double g1 = (al + 1.0) * (be + 1.0) / (al + be + 3.0) * g0;
  double p1 = ((al + be + 2.0) * x / 2.0 + (al - be) / 2.0) / std::sqrt(g1);
  if (n == 1) return p1;
  double aold = 2.0 / (2.0 + al + be) * std::sqrt((al + 1.0) * (be + 1.0) / (al + be + 3.0));
  double pm = p0, pc = p1;
  for (int i = 1; i < n; ++i) {
    double h1 = 2.0 * i + al + be;
    double anew = 2.0 / (h1 + 2.0) *
                  std::sqrt((i + 1.0) * (i + 1.0 + al + be) * (i + 1.0 + al) * (i + 1.0 + be) / (h1 + 1.0) / (h1 + 3.0));
    double bnew = -(al * al - be * be) / h1 / (h1 + 2.0);
    double pn = 1.0 / anew * (-aold * pm + (x - bnew) * pc);
    pm = pc;
    pc = pn;
    aold = anew;
  }
  return pc;
}

static double djacobi(double x, double al, double be, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + al + be + 1.0)) * jacobi(x, al + 1.0, be + 1.0, n - 1);
}

static void rst_to_abc(double r, double s, double t, double &a, double &b, double &c) {
  a = (std::fabs(s + t) > 1e-14) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
  b = (std::fabs(t - 1.0) > 1e-14) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
  c = t;
}

static inline double ipow(double x, int e) {
  double o = 1.0;
  for (int i = 0; i < e; ++i) o *= x;
  return o;
}

// orthonormal basis psi_{ijk} on the reference tetrahedron and its gradient
static void simplex3(double r, double s, double t, int i, int j, int k, double &v, double &dr, double &ds, double &dt) {
  double a, b, c;
  rst_to_abc(r, s, t, a, b, c);
  const double sc = 2.0 * std::sqrt(2.0);
  double A = jacobi(a, 0, 0, i), Ad = djacobi(a, 0, 0, i);
  double Pj = jacobi(b, 2.0 * i + 1.0, 0, j), Pjd = djacobi(b, 2.0 * i + 1.0, 0, j);
  double Pk = jacobi(c, 2.0 * (i + j) + 2.0, 0, k), Pkd = djacobi(c, 2.0 * (i + j) + 2.0, 0, k);
  double B = Pj * ipow(1.0 - b, i);
  double C = Pk * ipow(1.0 - c, i + j);
  double Bd = (i >= 1) ? Pj * ipow(1.0 - b, i - 1) : 0.0;          // B / (1-b)
  double Cd = (i + j >= 1) ? Pk * ipow(1.0 - c, i + j - 1) : 0.0;  // C / (1-c)
  double Bp = Pjd * ipow(1.0 - b, i) - ((i >= 1) ? i * Pj * ipow(1.0 - b, i - 1) : 0.0);
  double Cp = Pkd * ipow(1.0 - c, i + j) - ((i + j >= 1) ? (i + j) * Pk * ipow(1.0 - c, i + j - 1) : 0.0);
  v = sc * A * B * C;
  dr = sc * 4.0 * Ad * Bd * Cd;
  ds = sc * (2.0 * (1.0 + a) * Ad * Bd * Cd + 2.0 * A * Bp * Cd);
  dt = sc * (2.0 * (1.0 + a) * Ad * Bd * Cd + (1.0 + b) * A * Bp * Cd + A * B * Cp);
}

static double simplex2(double r, double s, int i, int j) {
  double a = (std::fabs(1.0 - s) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  double b = s;
  return std::sqrt(2.0) * jacobi(a, 0, 0, i) * jacobi(b, 2.0 * i + 1.0, 0, j) * ipow(1.0 - b, i);
}

// Gauss-Lobatto points of order N: -1, 1 and the roots of P_N' (Newton iteration)
static std::vector<double> lgl(int N) {
  std::vector<double> x(N + 1);
  for (int i = 0; i <= N; ++i) x[i] = -std::cos(M_PI * i / N);
  for (int i = 1; i < N; ++i) {
    double xi = x[i];
    for (int it = 0; it < 100; ++it) {
      // Legendre P_N, P_{N-1} by recurrence
      double p0 = 1.0, p1 = xi;
      for (int n = 2; n <= N; ++n) {
        double p2 = ((2.0 * n - 1.0) * xi * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
      }
      double PN = p1, PN1 = p0;
      double d1 = N * (PN1 - xi * PN) / (1.0 - xi * xi);           // P_N'
      double d2 = (2.0 * xi * d1 - N * (N + 1.0) * PN) / (1.0 - xi * xi);  // P_N''
      double dx = d1 / d2;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    x[i] = xi;
  }
  x[0] = -1.0;
  x[N] = 1.0;
  std::sort(x.begin(), x.end());
  return x;
}

static const double kAlphaOpt[15] = {0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603, 1.10153,
                                     0.6080, 0.4523, 0.8856, 0.8717, 0.9655};

// warp and blend node set (Warburton 2006), built on the equilateral tetrahedron
static void warp_blend(int N, const std::vector<int> &lat, std::vector<double> &r, std::vector<double> &s,
                       std::vector<double> &t) {
  const int Np = n_nodes(N);
  const double E[4][3] = {{-1.0, -1.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                          {1.0, -1.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                          {0.0, 2.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                          {0.0, 0.0, 3.0 / std::sqrt(6.0)}};
  const double alpha = kAlphaOpt[N - 1];
  const std::vector<double> xgl = lgl(N);
  std::vector<double> xeq(N + 1);
  for (int i = 0; i <= N; ++i) xeq[i] = -1.0 + 2.0 * i / N;
  // w(x)/(1-x^2) with w the 1-D warp (equispaced -> LGL)
  auto swarp = [&](double x) {
    double out = 0.0;
    for (int i = 1; i < N; ++i) {
      double term = (xgl[i] - xeq[i]) / (1.0 - xeq[i] * xeq[i]);
      for (int j = 1; j < N; ++j)
        if (j != i) term *= (x - xeq[j]) / (xeq[i] - xeq[j]);
      out += term;
    }
    return out;
  };
  const int faces[4][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {2, 0, 1, 3}, {3, 0, 1, 2}};  // a, then b c d
  r.assign(Np, 0);
  s.assign(Np, 0);
  t.assign(Np, 0);
  const double tol = 1e-10;
  for (int n = 0; n < Np; ++n) {
    double L[4];
    for (int q = 0; q < 4; ++q) L[q] = double(lat[n * 4 + q]) / N;
    double X[3] = {0, 0, 0}, sh[3] = {0, 0, 0};
    for (int q = 0; q < 4; ++q)
      for (int d = 0; d < 3; ++d) X[d] += L[q] * E[q][d];
    for (int f = 0; f < 4; ++f) {
      int a = faces[f][0], b = faces[f][1], c = faces[f][2], d4 = faces[f][3];
      double fw[3] = {0, 0, 0};
      const int edges[3][3] = {{b, c, d4}, {c, d4, b}, {d4, b, c}};
      for (auto &e : edges) {
        double x = L[e[1]] - L[e[0]];
        double amp = 4.0 * L[e[0]] * L[e[1]] * swarp(x) * (1.0 + (alpha * L[e[2]]) * (alpha * L[e[2]]));
        for (int d = 0; d < 3; ++d) fw[d] += amp * (E[e[1]][d] - E[e[0]][d]) / 2.0;
      }
      double La = L[a], Lb = L[b], Lc = L[c], Ld = L[d4];
      double blend = Lb * Lc * Ld;
      double den = (Lb + 0.5 * La) * (Lc + 0.5 * La) * (Ld + 0.5 * La);
      if (den > tol) blend = (1.0 + (alpha * La) * (alpha * La)) * blend / den;
      for (int d = 0; d < 3; ++d) sh[d] += blend * fw[d];
      int npos = (Lb > tol) + (Lc > tol) + (Ld > tol);
      if (La < tol && npos < 3)
        for (int d = 0; d < 3; ++d) sh[d] = fw[d];
    }
    for (int d = 0; d < 3; ++d) X[d] += sh[d];
    // barycentric coordinates on the equilateral tet: solve [E^T; 1] mu = [X; 1]
    std::vector<double> A(16);
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < 4; ++q) A[d * 4 + q] = E[q][d];
    for (int q = 0; q < 4; ++q) A[12 + q] = 1.0;
    invert(4, A);
    double rhs[4] = {X[0], X[1], X[2], 1.0}, mu[4];
    for (int q = 0; q < 4; ++q) {
      mu[q] = 0;
      for (int p = 0; p < 4; ++p) mu[q] += A[q * 4 + p] * rhs[p];
    }
    r[n] = 2.0 * mu[1] - 1.0;
    s[n] = 2.0 * mu[2] - 1.0;
    t[n] = 2.0 * mu[3] - 1.0;
  }
}

bool invert(int n, std::vector<double> &A) {
  // Gauss-Jordan with partial pivoting
  std::vector<double> B(n * n, 0.0);
  for (int i = 0; i < n; ++i) B[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(A[i * n + c]) > std::fabs(A[p * n + c])) p = i;
    if (A[p * n + c] == 0.0) return false;
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(A[p * n + j], A[c * n + j]);
        std::swap(B[p * n + j], B[c * n + j]);
      }
    double d = A[c * n + c];
    for (int j = 0; j < n; ++j) {
      A[c * n + j] /= d;
      B[c * n + j] /= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == c) continue;
      double f = A[i * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[i * n + j] -= f * A[c * n + j];
        B[i * n + j] -= f * B[c * n + j];
      }
    }
  }
  A = B;
  return true;
}

void basis_at(const RefOps &ref, double r, double s, double t, double *out) {
  int p = 0;
  double v, a, b, c;
  for (int i = 0; i <= ref.N; ++i)
    for (int j = 0; j <= ref.N - i; ++j)
      for (int k = 0; k <= ref.N - i - j; ++k) {
        simplex3(r, s, t, i, j, k, v, a, b, c);
        out[p++] = v;
      }
}

void build_ref(int N, RefOps &ref) {
  ref.N = N;
  const int Np = ref.Np = n_nodes(N);
  const int Nfp = ref.Nfp = n_face_nodes(N);
  ref.lat.clear();
  for (int l = 0; l <= N; ++l)
    for (int j = 0; j <= N - l; ++j)
      for (int i = 0; i <= N - l - j; ++i) {
        ref.lat.push_back(N - i - j - l);
        ref.lat.push_back(i);
        ref.lat.push_back(j);
        ref.lat.push_back(l);
      }
  warp_blend(N, ref.lat, ref.r, ref.s, ref.t);
  std::vector<double> V(Np * Np), Vr(Np * Np), Vs(Np * Np), Vt(Np * Np);
  for (int n = 0; n < Np; ++n) {
    int p = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j)
        for (int k = 0; k <= N - i - j; ++k) {
          simplex3(ref.r[n], ref.s[n], ref.t[n], i, j, k, V[n * Np + p], Vr[n * Np + p], Vs[n * Np + p],
                   Vt[n * Np + p]);
          ++p;
        }
  }
  ref.V = V;
  std::vector<double> Vi = V;
  invert(Np, Vi);
  auto mm = [&](const std::vector<double> &A, const std::vector<double> &B, int n, int k, int m) {
    std::vector<double> C(n * m, 0.0);
    for (int i = 0; i < n; ++i)
      for (int q = 0; q < k; ++q) {
        double a = A[i * k + q];
        for (int j = 0; j < m; ++j) C[i * m + j] += a * B[q * m + j];
      }
    return C;
  };
  ref.Dr = mm(Vr, Vi, Np, Np, Np);
  ref.Ds = mm(Vs, Vi, Np, Np, Np);
  ref.Dt = mm(Vt, Vi, Np, Np, Np);
  // face nodes: barycentric weight of the opposite vertex is zero
  ref.Fmask.assign(4 * Nfp, 0);
  for (int f = 0; f < 4; ++f) {
    int c = 0;
    for (int n = 0; n < Np; ++n)
      if (ref.lat[n * 4 + kFaceOpp[f]] == 0) ref.Fmask[f * Nfp + c++] = n;
  }
  // face mass matrices from the 2-D orthonormal basis on each face's two free coordinates
  std::vector<double> Emat(Np * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    std::vector<double> V2(Nfp * Nfp);
    for (int i = 0; i < Nfp; ++i) {
      int n = ref.Fmask[f * Nfp + i];
      double u, v;
      if (f == 0) { u = ref.r[n]; v = ref.s[n]; }
      else if (f == 1) { u = ref.r[n]; v = ref.t[n]; }
      else if (f == 2) { u = ref.s[n]; v = ref.t[n]; }
      else { u = ref.s[n]; v = ref.t[n]; }
      int p = 0;
      for (int a = 0; a <= N; ++a)
        for (int b = 0; b <= N - a; ++b) V2[i * Nfp + p++] = simplex2(u, v, a, b);
    }
    // M_f = (V2 V2^T)^{-1}
    std::vector<double> MM(Nfp * Nfp, 0.0);
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j) {
        double acc = 0;
        for (int p = 0; p < Nfp; ++p) acc += V2[i * Nfp + p] * V2[j * Nfp + p];
        MM[i * Nfp + j] = acc;
      }
    invert(Nfp, MM);
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j) Emat[ref.Fmask[f * Nfp + i] * (4 * Nfp) + f * Nfp + j] = MM[i * Nfp + j];
  }
  // LIFT = V (V^T E)
  std::vector<double> Vt_(Np * Np);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) Vt_[i * Np + j] = V[j * Np + i];
  ref.LIFT = mm(V, mm(Vt_, Emat, Np, Np, 4 * Nfp), Np, Np, 4 * Nfp);
  // face node matching tables (combinatorial, by barycentric weights on shared vertices)
  ref.nbr_index.assign(4 * 4 * 6 * Nfp, -1);
  for (int f = 0; f < 4; ++f)
    for (int f2 = 0; f2 < 4; ++f2)
      for (int p = 0; p < 6; ++p)
        for (int i = 0; i < Nfp; ++i) {
          int n = ref.Fmask[f * Nfp + i];
          int want[3];
          for (int a = 0; a < 3; ++a) want[kPerm3[p][a]] = ref.lat[n * 4 + kFaceVerts[f][a]];
          for (int i2 = 0; i2 < Nfp; ++i2) {
            int n2 = ref.Fmask[f2 * Nfp + i2];
            bool ok = true;
            for (int u = 0; u < 3; ++u) ok = ok && ref.lat[n2 * 4 + kFaceVerts[f2][u]] == want[u];
            if (ok) {
              ref.nbr_index[((f * 4 + f2) * 6 + p) * Nfp + i] = i2;
              break;
            }
          }
        }
}

// ---------------------------------------------------------------------------------------------
// mesh
// ---------------------------------------------------------------------------------------------
std::string mesh_build(HostMesh &m, int N, int64_t n_vert, const double *xyz, int64_t K, const int64_t *etov,
                       const int8_t *face_bc, int bc_default, const RefOps &ref) {
  (void)ref;
  m.N = N;
  m.K = K;
  m.n_vert = n_vert;
  m.verts.assign(xyz, xyz + 3 * n_vert);
  m.etov.assign(etov, etov + 4 * K);
  m.geo.assign(9 * K, 0.0);
  m.J.assign(K, 0.0);
  for (int64_t k = 0; k < K; ++k) {
    for (int a = 0; a < 4; ++a)
      if (m.etov[4 * k + a] < 0 || m.etov[4 * k + a] >= n_vert) return "vertex index out of range";
    const double *v[4];
    for (int a = 0; a < 4; ++a) v[a] = &m.verts[3 * m.etov[4 * k + a]];
    double e1[3], e2[3], e3[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = v[1][d] - v[0][d];
      e2[d] = v[2][d] - v[0][d];
      e3[d] = v[3][d] - v[0][d];
    }
    double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) + e1[1] * (e2[2] * e3[0] - e2[0] * e3[2]) +
                 e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    if (!(det != 0.0) || !std::isfinite(det)) return "degenerate element";
    if (det < 0) {
      std::swap(m.etov[4 * k + 2], m.etov[4 * k + 3]);
      for (int a = 0; a < 4; ++a) v[a] = &m.verts[3 * m.etov[4 * k + a]];
    }
    // A = [x_r x_s x_t] = [(v1-v0)/2 (v2-v0)/2 (v3-v0)/2]; rows of A^{-1} are grad r, grad s, grad t
    double A[3][3];
    for (int d = 0; d < 3; ++d) {
      A[d][0] = 0.5 * (v[1][d] - v[0][d]);
      A[d][1] = 0.5 * (v[2][d] - v[0][d]);
      A[d][2] = 0.5 * (v[3][d] - v[0][d]);
    }
    double J = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(J > 0.0)) return "non-positive Jacobian";
    m.J[k] = J;
    double inv[3][3];
    inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / J;
    inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / J;
    inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / J;
    inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / J;
    inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / J;
    inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / J;
    inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / J;
    inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / J;
    inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / J;
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) m.geo[9 * k + 3 * j + i] = inv[j][i];
  }
  // faces: key = sorted global vertex triple; match by sorting
  struct FaceRec {
    std::array<int64_t, 3> key;
    int64_t k;
    int f;
  };
  std::vector<FaceRec> fr(4 * K);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      std::array<int64_t, 3> key = {m.etov[4 * k + kFaceVerts[f][0]], m.etov[4 * k + kFaceVerts[f][1]],
                                    m.etov[4 * k + kFaceVerts[f][2]]};
      std::sort(key.begin(), key.end());
      fr[4 * k + f] = {key, k, f};
    }
  std::sort(fr.begin(), fr.end(), [](const FaceRec &a, const FaceRec &b) {
    if (a.key != b.key) return a.key < b.key;
    if (a.k != b.k) return a.k < b.k;
    return a.f < b.f;
  });
  m.EToE.assign(4 * K, 0);
  m.EToF.assign(4 * K, 0);
  m.face_perm.assign(4 * K, 0);
  m.bc.assign(4 * K, 0);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      m.EToE[4 * k + f] = (int32_t)k;
      m.EToF[4 * k + f] = (int8_t)f;
    }
  for (size_t i = 0; i < fr.size();) {
    size_t j = i + 1;
    while (j < fr.size() && fr[j].key == fr[i].key) ++j;
    if (j - i > 2) return "non-manifold face";
    if (j - i == 2) {
      const FaceRec &a = fr[i], &b = fr[i + 1];
      m.EToE[4 * a.k + a.f] = (int32_t)b.k;
      m.EToF[4 * a.k + a.f] = (int8_t)b.f;
      m.EToE[4 * b.k + b.f] = (int32_t)a.k;
      m.EToF[4 * b.k + b.f] = (int8_t)a.f;
      for (int side = 0; side < 2; ++side) {
        const FaceRec &x = side ? b : a, &y = side ? a : b;
        int64_t G[3], H[3];
        for (int t = 0; t < 3; ++t) {
          G[t] = m.etov[4 * x.k + kFaceVerts[x.f][t]];
          H[t] = m.etov[4 * y.k + kFaceVerts[y.f][t]];
        }
        int code = -1;
        for (int p = 0; p < 6 && code < 0; ++p) {
          bool ok = true;
          for (int t = 0; t < 3; ++t) ok = ok && G[t] == H[kPerm3[p][t]];
          if (ok) code = p;
        }
        if (code < 0) return "face vertex mismatch";
        m.face_perm[4 * x.k + x.f] = (int8_t)code;
      }
    } else {
      const FaceRec &a = fr[i];
      int b = face_bc ? face_bc[4 * a.k + a.f] : bc_default;
      if (b < 1 || b > 3) return "boundary face without a valid boundary type";
      m.bc[4 * a.k + a.f] = (int8_t)b;
    }
    i = j;
  }
  m.has_model = false;
  return "";
}

std::string mesh_set_model(HostMesh &m, const double *rho, const double *c, int n_levels_max, double cfl) {
  const int64_t K = m.K;
  if (n_levels_max < 1 || n_levels_max > 8) return "n_levels_max must be in 1..8";
  m.rho.assign(rho, rho + K);
  m.c.assign(c, c + K);
  for (int64_t k = 0; k < K; ++k)
    if (!(m.rho[k] > 0) || !(m.c[k] > 0)) return "rho and c must be positive";
  // dt_k = cfl * l_k / ((N+1)^2 c_k), l_k = 3 V_k / max face area (fixed operation order)
  std::vector<double> dt(K);
  const double np2 = double((m.N + 1) * (m.N + 1));
  for (int64_t k = 0; k < K; ++k) {
    const double *v[4];
    for (int a = 0; a < 4; ++a) v[a] = &m.verts[3 * m.etov[4 * k + a]];
    double e1[3], e2[3], e3[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = v[1][d] - v[0][d];
      e2[d] = v[2][d] - v[0][d];
      e3[d] = v[3][d] - v[0][d];
    }
    double cx = e2[1] * e3[2] - e2[2] * e3[1];
    double cy = e2[2] * e3[0] - e2[0] * e3[2];
    double cz = e2[0] * e3[1] - e2[1] * e3[0];
    double vol = std::fabs(e1[0] * cx + e1[1] * cy + e1[2] * cz) / 6.0;
    double amax = 0.0;
    for (int f = 0; f < 4; ++f) {
      const double *a = v[kFaceVerts[f][0]], *b = v[kFaceVerts[f][1]], *cc = v[kFaceVerts[f][2]];
      double f1[3], f2[3];
      for (int d = 0; d < 3; ++d) {
        f1[d] = b[d] - a[d];
        f2[d] = cc[d] - a[d];
      }
      double gx = f1[1] * f2[2] - f1[2] * f2[1];
      double gy = f1[2] * f2[0] - f1[0] * f2[2];
      double gz = f1[0] * f2[1] - f1[1] * f2[0];
      double area = 0.5 * std::sqrt(gx * gx + gy * gy + gz * gz);
      amax = std::max(amax, area);
    }
    double ell = 3.0 * vol / amax;
    dt[k] = cfl * ell / (np2 * m.c[k]);
  }
  double dtl = *std::min_element(dt.begin(), dt.end());
  int L = n_levels_max;
  std::vector<int> lev(K, L);
  for (int64_t k = 0; k < K; ++k)
    for (int l = L; l >= 1; --l)
      if (std::ldexp(1.0, L - l) * dtl <= dt[k]) lev[k] = l;
  // neighbours differ by at most one level: raise levels to a fixed point
  bool changed = true;
  while (changed) {
    changed = false;
    std::vector<int> nl(lev);
    for (int64_t k = 0; k < K; ++k) {
      int mx = lev[k];
      for (int f = 0; f < 4; ++f) mx = std::max(mx, lev[m.EToE[4 * k + f]] - 1);
      nl[k] = mx;
    }
    for (int64_t k = 0; k < K; ++k)
      if (nl[k] != lev[k]) changed = true;
    lev.swap(nl);
  }
  while (L > 1) {
    bool any1 = false;
    for (int64_t k = 0; k < K && !any1; ++k) any1 = lev[k] == 1;
    if (any1) break;
    for (auto &x : lev) --x;
    --L;
  }
  m.L = L;
  m.dt_local = dtl;
  m.level.assign(K, 0);
  for (int64_t k = 0; k < K; ++k) m.level[k] = (int8_t)lev[k];
  // level-sorted layout, finest level first, user order inside a level, segments padded to 64
  m.lev_begin.assign(L + 1, 0);
  m.lev_count.assign(L + 1, 0);
  for (int64_t k = 0; k < K; ++k) m.lev_count[lev[k] - 1]++;
  int64_t pos = 0;
  std::vector<int64_t> begin(L, 0);
  for (int l = L; l >= 1; --l) {
    begin[l - 1] = pos;
    pos += (m.lev_count[l - 1] + 63) / 64 * 64;
  }
  m.Ktot = pos;
  for (int l = 0; l < L; ++l) m.lev_begin[l] = begin[l];
  m.lev_begin[L] = pos;
  m.sorted_to_user.assign(m.Ktot, -1);
  m.user_to_sorted.assign(K, -1);
  std::vector<int64_t> fill(begin);
  for (int64_t k = 0; k < K; ++k) {
    int64_t s = fill[lev[k] - 1]++;
    m.sorted_to_user[s] = k;
    m.user_to_sorted[k] = s;
  }
  m.has_model = true;
  return "";
}

void mesh_vmapP(const HostMesh &m, const RefOps &ref, int32_t *vmapP) {
  const int Np = ref.Np, Nfp = ref.Nfp;
  for (int64_t k = 0; k < m.K; ++k)
    for (int f = 0; f < 4; ++f) {
      int64_t k2 = m.EToE[4 * k + f];
      int f2 = m.EToF[4 * k + f];
      int p = m.face_perm[4 * k + f];
      for (int i = 0; i < Nfp; ++i) {
        int64_t out;
        if (k2 == k && f2 == f && m.bc[4 * k + f] != 0) {
          out = k * Np + ref.Fmask[f * Nfp + i];
        } else {
          int i2 = ref.nbr_index[((f * 4 + f2) * 6 + p) * Nfp + i];
          out = k2 * Np + ref.Fmask[f2 * Nfp + i2];
        }
        vmapP[(k * 4 + f) * Nfp + i] = (int32_t)out;
      }
    }
}

void locate_points(const HostMesh &m, int64_t n, const double *xyz, int64_t *elem, double *rst) {
  const int64_t K = m.K;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < m.n_vert; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], m.verts[3 * i + d]);
      hi[d] = std::max(hi[d], m.verts[3 * i + d]);
    }
  // bucket grid with about one element per bucket
  int nb = std::max<int64_t>(1, (int64_t)std::cbrt((double)K / 6.0));
  double w[3];
  for (int d = 0; d < 3; ++d) w[d] = (hi[d] - lo[d]) / nb + 1e-300;
  auto cell = [&](double x, int d) {
    int c = (int)std::floor((x - lo[d]) / w[d]);
    return std::min(std::max(c, 0), nb - 1);
  };
  std::vector<std::vector<int64_t>> buckets((size_t)nb * nb * nb);
  for (int64_t k = 0; k < K; ++k) {
    double a[3] = {1e300, 1e300, 1e300}, b[3] = {-1e300, -1e300, -1e300};
    for (int q = 0; q < 4; ++q)
      for (int d = 0; d < 3; ++d) {
        double x = m.verts[3 * m.etov[4 * k + q] + d];
        a[d] = std::min(a[d], x);
        b[d] = std::max(b[d], x);
      }
    for (int i = cell(a[0] - 1e-9, 0); i <= cell(b[0] + 1e-9, 0); ++i)
      for (int j = cell(a[1] - 1e-9, 1); j <= cell(b[1] + 1e-9, 1); ++j)
        for (int l = cell(a[2] - 1e-9, 2); l <= cell(b[2] + 1e-9, 2); ++l)
          buckets[((size_t)l * nb + j) * nb + i].push_back(k);
  }
  for (int64_t p = 0; p < n; ++p) {
    const double *x = xyz + 3 * p;
    elem[p] = -1;
    const auto &cand = buckets[((size_t)cell(x[2], 2) * nb + cell(x[1], 1)) * nb + cell(x[0], 0)];
    for (int64_t k : cand) {  // candidates are in increasing element order
      if (elem[p] >= 0 && k > elem[p]) break;
      const double *v0 = &m.verts[3 * m.etov[4 * k]];
      // lambda_{1..3} = grad (r,s,t) . (x - v0) written through the inverse metric: r+1 = 2 lambda_1
      double d[3] = {x[0] - v0[0], x[1] - v0[1], x[2] - v0[2]};
      double lam[4];
      for (int j = 0; j < 3; ++j) {
        const double *g = &m.geo[9 * k + 3 * j];
        lam[j + 1] = 0.5 * (g[0] * d[0] + g[1] * d[1] + g[2] * d[2]);
      }
      lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
      bool in = lam[0] >= -1e-12 && lam[1] >= -1e-12 && lam[2] >= -1e-12 && lam[3] >= -1e-12;
      if (in) {
        elem[p] = k;
        rst[3 * p + 0] = 2.0 * lam[1] - 1.0;
        rst[3 * p + 1] = 2.0 * lam[2] - 1.0;
        rst[3 * p + 2] = 2.0 * lam[3] - 1.0;
      }
    }
  }
}

}  // namespace dgrtm
