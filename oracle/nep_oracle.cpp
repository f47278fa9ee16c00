// FP64 CPU oracle of the NEP molecular-dynamics evaluation.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library. It shares no code, header,
// table or constant with the HIP library.
//
// It is a plain, slow, direct statement of what the method computes:
//   * the atomic energy of the single-hidden-layer network (Section III.B, the
//     equation for U_i), summed to the total energy;
//   * radial descriptors q_n = sum_j g_n(r_ij) and angular descriptors q_nl from
//     radial functions times spherical harmonics contracted over m
//     (Section III.B), with Chebyshev first-kind radial bases (Section III.B)
//     and separate radial / angular cutoffs (Fig. 1);
//   * the four-body term with l_max = 2 (Section VI.A);
//   * optionally, the ZBL screened-Coulomb repulsion added to the Cu and HfO2
//     models (Section VI.A), half of each pair's energy per atom;
//   * forces F = -dU/dx and the virial;
//   * velocity-Verlet integration with the step, temperature and neighbour
//     settings of Section VI.A, and its NVT form with a Nose-Hoover chain (the
//     application run of Section VII uses the NVT ensemble);
//   * gradients of energy and force losses with respect to the network weights.
//
// Where the paper names a piece without printing its formula, this file takes
// the published NEP forms (reference [8] of the paper):
//   f_c(r) = (1 + cos(pi r / r_c)) / 2 for r < r_c, else 0
//   x = 2 (r / r_c - 1)^2 - 1,  T_0 = 1, T_1 = x, T_{k+1} = 2 x T_k - T_{k-1}
//   f_k(r) = (T_k(x) + 1) f_c(r) / 2,  g_n(r) = sum_k c^{t_i t_j}_{nk} f_k(r)
//   q_nl = (4 pi / (2l+1)) sum_m s_nlm^2 = sum_{j,k} g_n(r_ij) g_n(r_ik) P_l(cos theta_jk)
//   four-body: S_n = sum_j g_n(r_ij) (u u^T - I/3),  q4_n = tr(S_n^3)
// Descriptor order: [radial n | angular, l-major then n | four-body n].
// Build: g++ -O2 -ffp-contract=off -fopenmp (no fast-math, no FMA contraction).
//
// Parity pins: every function here is checked in the CPU test suite against closed
// forms, library routines, brute force, invariances or finite differences, with one
// partial exception. The ZBL term's universal screening constants (the four weights
// c_m and exponents d_m, the 0.8854 a_0 screening length and the 0.23 power, from
// J. F. Ziegler, J. P. Biersack and U. Littmark, "The Stopping and Range of Ions in
// Solids", Pergamon, 1985) are PARITY UNPINNED as values: the tests fix the weights'
// sum (the bare-Coulomb limit r -> 0), the switch, and forces and virial against
// central differences, but a mistyped exponent or screening length would pass them,
// since neither the paper nor any fixture here prints the function's values.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;
const double kXi = 103.642697;          // eV per (amu A^2 / fs^2)
const double kBoltzmann = 8.617333262e-5;  // eV / K

enum { OK = 0, ERR_ARG = -1, ERR_BOX = -2, ERR_CAP = -3 };

struct Model {
  int T = 0, nR = 0, kR = 0, nA = 0, kA = 0, L3 = 0, L4 = 0, H = 0, D = 0;
  double rcR = 0, rcA = 0;
  double zi = 0, zo = 0;        // ZBL switching radii (zo = 0: no ZBL term)
  double Z[2] = {0, 0};         // atomic number of each species (ZBL)
  const double* cR = nullptr;   // [T][T][nR][kR]
  const double* cA = nullptr;   // [T][T][nA][kA]
  const double* sigma = nullptr;  // [D]
  const double* W0 = nullptr;   // [H][D]
  const double* b0 = nullptr;   // [H]
  const double* w1 = nullptr;   // [H]
  double b1 = 0;
  int64_t n_params = 0;
  int64_t off_nn = 0;  // offset of W0 in the packed vector
};

// ip = {n_types, n_max_R, n_max_A, basis_R, basis_A, l_max_3b, l_max_4b, n_hidden}
// dp = {rc_radial, rc_angular, zbl_inner, zbl_outer, Z_0, Z_1}
int parse_model(const int32_t* ip, const double* dp, const double* p, int64_t n_params, Model& m) {
  if (!ip || !dp || !p) return ERR_ARG;
  m.T = ip[0];
  m.nR = ip[1] + 1;
  m.nA = ip[2] + 1;
  m.kR = ip[3] + 1;
  m.kA = ip[4] + 1;
  m.L3 = ip[5];
  m.L4 = ip[6];
  m.H = ip[7];
  m.rcR = dp[0];
  m.rcA = dp[1];
  if (m.T < 1 || m.nR < 1 || m.nA < 1 || m.kR < 2 || m.kA < 2 || m.L3 < 1 || m.L3 > 8 ||
      !(m.L4 == 0 || m.L4 == 2) || m.H < 1 || !(m.rcR > 0) || !(m.rcA > 0) || m.rcA > m.rcR)
    return ERR_ARG;
  m.zi = dp[2];
  m.zo = dp[3];
  m.Z[0] = dp[4];
  m.Z[1] = dp[5];
  if (m.zo != 0.0) {
    if (!(m.zo > 0 && m.zi >= 0 && m.zi < m.zo && m.zo <= m.rcR) || m.T > 2) return ERR_ARG;
    for (int t = 0; t < m.T; ++t)
      if (!(m.Z[t] > 0)) return ERR_ARG;
  }
  m.D = m.nR + m.nA * m.L3 + (m.L4 == 2 ? m.nA : 0);
  int64_t off = 0;
  m.cR = p + off; off += (int64_t)m.T * m.T * m.nR * m.kR;
  m.cA = p + off; off += (int64_t)m.T * m.T * m.nA * m.kA;
  m.sigma = p + off; off += m.D;
  m.off_nn = off;
  m.W0 = p + off; off += (int64_t)m.H * m.D;
  m.b0 = p + off; off += m.H;
  m.w1 = p + off; off += m.H;
  m.b1 = p[off]; off += 1;
  m.n_params = off;
  if (off != n_params) return ERR_ARG;
  return OK;
}

// ------------------------------------------------------------------ geometry
// Minimum-image difference and squared distance, written exactly as
//   d = x_j - x_i; if (d > L/2) d -= L; else if (d < -L/2) d += L;
//   r2 = (dx*dx + dy*dy) + dz*dz
void min_image(const double* box, double* d) {
  for (int c = 0; c < 3; ++c) {
    const double half = 0.5 * box[c];
    if (d[c] > half) d[c] -= box[c];
    else if (d[c] < -half) d[c] += box[c];
  }
}

double r2_of(const double* d) {
  double s = d[0] * d[0];
  s = s + d[1] * d[1];
  s = s + d[2] * d[2];
  return s;
}

void pair_vec(const double* x, const double* box, int64_t i, int64_t j, double* d) {
  d[0] = x[3 * j + 0] - x[3 * i + 0];
  d[1] = x[3 * j + 1] - x[3 * i + 1];
  d[2] = x[3 * j + 2] - x[3 * i + 2];
  min_image(box, d);
}

// Cell list used only to find candidate pairs; membership is decided by r2 < cut^2.
struct CellGrid {
  int nc[3] = {1, 1, 1};
  std::vector<int64_t> head;  // start offsets, size ncell+1
  std::vector<int64_t> atoms; // atom ids grouped by cell, ascending within a cell
  int cell_coord(double xv, double L, int n) const {
    double w = xv - L * std::floor(xv / L);
    int c = (int)std::floor(w / L * n);
    if (c < 0) c = 0;
    if (c >= n) c = n - 1;
    return c;
  }
  void build(int64_t n, const double* x, const double* box, double cut) {
    for (int c = 0; c < 3; ++c) {
      nc[c] = (int)std::floor(box[c] / cut);
      if (nc[c] < 1) nc[c] = 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    std::vector<int64_t> cid(n);
    std::vector<int64_t> cnt(ncell + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      int cx = cell_coord(x[3 * i + 0], box[0], nc[0]);
      int cy = cell_coord(x[3 * i + 1], box[1], nc[1]);
      int cz = cell_coord(x[3 * i + 2], box[2], nc[2]);
      cid[i] = ((int64_t)cz * nc[1] + cy) * nc[0] + cx;
      cnt[cid[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cnt[c + 1] += cnt[c];
    head = cnt;
    atoms.assign(n, 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i) atoms[fill[cid[i]]++] = i;
  }
  // Distinct neighbour cells of the cell holding atom i.
  void neighbor_cells(const double* x, const double* box, int64_t i, std::vector<int64_t>& out) const {
    int c0[3];
    for (int c = 0; c < 3; ++c) c0[c] = cell_coord(x[3 * i + c], box[c], nc[c]);
    int offs[3][3];
    int noff[3];
    for (int c = 0; c < 3; ++c) {
      if (nc[c] >= 3) { offs[c][0] = -1; offs[c][1] = 0; offs[c][2] = 1; noff[c] = 3; }
      else if (nc[c] == 2) { offs[c][0] = 0; offs[c][1] = 1; noff[c] = 2; }
      else { offs[c][0] = 0; noff[c] = 1; }
    }
    out.clear();
    for (int a = 0; a < noff[2]; ++a)
      for (int b = 0; b < noff[1]; ++b)
        for (int e = 0; e < noff[0]; ++e) {
          int cx = (c0[0] + offs[0][e] + nc[0]) % nc[0];
          int cy = (c0[1] + offs[1][b] + nc[1]) % nc[1];
          int cz = (c0[2] + offs[2][a] + nc[2]) % nc[2];
          out.push_back(((int64_t)cz * nc[1] + cy) * nc[0] + cx);
        }
  }
};

// Neighbours of atom i with r2 < cut^2, ascending by id.
void neighbors_of(const CellGrid* g, int64_t n, const double* x, const double* box, double cut,
                  int64_t i, std::vector<int32_t>& out) {
  out.clear();
  const double cut2 = cut * cut;
  double d[3];
  if (!g) {
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      pair_vec(x, box, i, j, d);
      if (r2_of(d) < cut2) out.push_back((int32_t)j);
    }
    return;
  }
  std::vector<int64_t> cells;
  g->neighbor_cells(x, box, i, cells);
  for (int64_t c : cells)
    for (int64_t p = g->head[c]; p < g->head[c + 1]; ++p) {
      int64_t j = g->atoms[p];
      if (j == i) continue;
      pair_vec(x, box, i, j, d);
      if (r2_of(d) < cut2) out.push_back((int32_t)j);
    }
  std::sort(out.begin(), out.end());
}

bool box_ok(const double* box, double cut) {
  for (int c = 0; c < 3; ++c)
    if (!(box[c] >= 2.0 * cut)) return false;
  return true;
}

// ------------------------------------------------------------------ bases
// f_k(r) and df_k/dr for k = 0..K-1 (Chebyshev-based radial basis times cutoff).
void radial_basis(double r, double rc, int K, double* f, double* df) {
  for (int k = 0; k < K; ++k) { f[k] = 0; df[k] = 0; }
  if (!(r < rc)) return;
  const double fc = 0.5 * (1.0 + std::cos(kPi * r / rc));
  const double dfc = -0.5 * kPi / rc * std::sin(kPi * r / rc);
  const double y = r / rc - 1.0;
  const double xx = 2.0 * y * y - 1.0;
  const double dx = 4.0 * y / rc;
  std::vector<double> T(K), dT(K);
  T[0] = 1.0; dT[0] = 0.0;
  if (K > 1) { T[1] = xx; dT[1] = 1.0; }
  for (int k = 2; k < K; ++k) {
    T[k] = 2.0 * xx * T[k - 1] - T[k - 2];
    dT[k] = 2.0 * T[k - 1] + 2.0 * xx * dT[k - 1] - dT[k - 2];
  }
  for (int k = 0; k < K; ++k) {
    f[k] = 0.5 * (T[k] + 1.0) * fc;
    df[k] = 0.5 * dT[k] * dx * fc + 0.5 * (T[k] + 1.0) * dfc;
  }
}

// Legendre P_l(c) and P_l'(c), l = 0..L (Bonnet recurrence; derivative recurrence
// P'_{l+1} = P'_{l-1} + (2l+1) P_l, regular at c = +-1).
void legendre(double c, int L, double* P, double* dP) {
  P[0] = 1.0; dP[0] = 0.0;
  if (L >= 1) { P[1] = c; dP[1] = 1.0; }
  for (int l = 1; l < L; ++l) {
    P[l + 1] = ((2.0 * l + 1.0) * c * P[l] - l * P[l - 1]) / (l + 1.0);
    dP[l + 1] = dP[l - 1] + (2.0 * l + 1.0) * P[l];
  }
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Real orthonormal spherical harmonics Y_lm(u), m = -l..l stored at [m + l], built
// from associated Legendre functions (no Condon-Shortley phase) and cos/sin(m phi).
void real_sph_harm(int l, const double* u, double* Y) {
  const double ct = std::max(-1.0, std::min(1.0, u[2]));
  const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  const double phi = std::atan2(u[1], u[0]);
  for (int m = 0; m <= l; ++m) {
    // P_l^m(ct) by upward recurrence in l from P_m^m.
    double pmm = 1.0;
    for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * st;
    double plm;
    if (l == m) plm = pmm;
    else {
      double pm1 = ct * (2.0 * m + 1.0) * pmm;
      if (l == m + 1) plm = pm1;
      else {
        double a = pmm, b = pm1, cval = 0;
        for (int ll = m + 2; ll <= l; ++ll) {
          cval = ((2.0 * ll - 1.0) * ct * b - (ll + m - 1.0) * a) / (ll - m);
          a = b; b = cval;
        }
        plm = cval;
      }
    }
    const double norm = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * factorial(l - m) / factorial(l + m));
    if (m == 0) Y[l] = norm * plm;
    else {
      Y[l + m] = std::sqrt(2.0) * norm * plm * std::cos(m * phi);
      Y[l - m] = std::sqrt(2.0) * norm * plm * std::sin(m * phi);
    }
  }
}

// ZBL universal screened Coulomb repulsion between species ti and tj at distance r
// (Ziegler, Biersack and Littmark; Section VI.A adds it to the Cu and HfO2 models
// with an outer cutoff):
//   phi(r) = k_e Z_i Z_j / r * sum_m c_m exp(-d_m r / a),  a = 0.8854 a_0 / (Z_i^0.23 + Z_j^0.23),
// with k_e = e^2 / (4 pi eps_0) and a_0 the Bohr radius, multiplied by a switch that
// is 1 below zi, (1 + cos(pi (r - zi) / (zo - zi))) / 2 between zi and zo and 0 beyond.
// Returns the switched energy e and its derivative de = d e / d r.
void zbl_pair(const Model& m, int ti, int tj, double r, double& e, double& de) {
  e = 0.0;
  de = 0.0;
  if (!(m.zo > 0.0) || !(r < m.zo)) return;
  const double ke = 14.399645478;   // eV A
  const double a0 = 0.529177210903;  // A
  const double c[4] = {0.18175, 0.50986, 0.28022, 0.02817};
  const double d[4] = {3.19980, 0.94229, 0.40290, 0.20162};
  const double zz = m.Z[ti] * m.Z[tj];
  const double a = 0.8854 * a0 / (std::pow(m.Z[ti], 0.23) + std::pow(m.Z[tj], 0.23));
  double S = 0.0, dS = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double t = c[k] * std::exp(-d[k] * r / a);
    S += t;
    dS += -d[k] / a * t;
  }
  const double phi = ke * zz / r * S;
  const double dphi = ke * zz * (dS / r - S / (r * r));
  double sw = 1.0, dsw = 0.0;
  if (r >= m.zi) {
    const double w = kPi / (m.zo - m.zi);
    sw = 0.5 * (1.0 + std::cos(w * (r - m.zi)));
    dsw = -0.5 * w * std::sin(w * (r - m.zi));
  }
  e = phi * sw;
  de = dphi * sw + phi * dsw;
}

// Round to bfloat16 (8 significant bits) with round-to-nearest-even, from FP64.
double round_bf16(double v) {
  if (v == 0.0 || !std::isfinite(v)) return v;
  int e = 0;
  const double m = std::frexp(v, &e);      // |m| in [0.5, 1)
  const double s = std::ldexp(m, 8);       // |s| in [128, 256)
  const double r = std::nearbyint(s);      // default rounding mode: nearest-even
  return std::ldexp(r, e - 8);
}

// Network of Section III.B on one descriptor vector q [D]:
//   U = sum_mu w1_mu tanh(h_mu) - b1,  h = W0 q~ - b0,  q~ = q * sigma,
//   Fp = dU/dq = sigma * W0^T (w1 * (1 - tanh^2 h)),
// with h [H] returned too. bf16 != 0 is the bfloat16 form: q~, W0 and w1 (1 - tanh^2 h)
// are rounded to bfloat16 before the products that use them (FP64 accumulation).
void network(const Model& m, const double* q, int bf16, double& U, std::vector<double>& Fp,
             std::vector<double>& h) {
  const int D = m.D, H = m.H;
  std::vector<double> qs(D), Wr(H * D);
  for (int v = 0; v < D; ++v) qs[v] = q[v] * m.sigma[v];
  for (int k = 0; k < H * D; ++k) Wr[k] = m.W0[k];
  if (bf16) {
    for (int v = 0; v < D; ++v) qs[v] = round_bf16(qs[v]);
    for (int k = 0; k < H * D; ++k) Wr[k] = round_bf16(Wr[k]);
  }
  h.assign(H, 0.0);
  std::vector<double> a1(H);
  U = 0;
  for (int mu = 0; mu < H; ++mu) {
    double s = 0;
    for (int v = 0; v < D; ++v) s += Wr[mu * D + v] * qs[v];
    const double hh = s - m.b0[mu];
    h[mu] = hh;
    const double t = std::tanh(hh);
    U += m.w1[mu] * t;
    a1[mu] = m.w1[mu] * (1.0 - t * t);
    if (bf16) a1[mu] = round_bf16(a1[mu]);
  }
  U -= m.b1;
  Fp.assign(D, 0.0);
  for (int v = 0; v < D; ++v) {
    double s = 0;
    for (int mu = 0; mu < H; ++mu) s += Wr[mu * D + v] * a1[mu];
    Fp[v] = m.sigma[v] * s;
  }
}

// ------------------------------------------------------------------ per-center terms
struct PairGeom {
  int32_t j;
  double d[3];  // r_ij = x_j - x_i (minimum image)
  double r;
  double u[3];
};

// Everything one center contributes: its descriptor, energy, dU/dq and, for each
// radial neighbour j, the descriptor Jacobian dq/dr_ij (D x 3).
struct CenterTerms {
  std::vector<double> q;    // [D]
  double U = 0;
  std::vector<double> h;    // [H] hidden pre-activation
  std::vector<double> Fp;   // [D] dU/dq (unscaled descriptor)
  std::vector<PairGeom> pairs;  // radial neighbours (r < rcR), ascending id
  std::vector<double> J;    // [npairs][D][3] dq_nu / d r_ij
  std::vector<double> zd;   // [npairs] d(half the ZBL pair energy)/dr (zero without ZBL)
};

// Intermediate per-pair tables of one center, kept on request for the
// coefficient gradients: basis values f_k, df_k/dr at both cutoffs, the angular
// radial functions g_n and g_n', the angular pair indices, the Legendre tables
// over angular pairs and the four-body matrices S_n.
struct CenterTables {
  std::vector<double> fR, dfR;   // [npairs][kR]
  std::vector<double> fA, dfA;   // [npairs][kA] (zero beyond the angular cutoff)
  std::vector<double> gA, dgA;   // [npairs][nA]
  std::vector<int> ang;          // pair index of each angular neighbour
  std::vector<double> cosjk, Pjk, dPjk;  // [na][na], [na][na][L3+1] x 2
  std::vector<double> S;         // [nA][3][3]
};

// jac_for: -2 = no Jacobian, -1 = every pair, >= 0 = only the pair with that neighbour id.
void center_terms(const Model& m, const CellGrid* g, int64_t n, const double* x, const int32_t* type,
                  const double* box, int64_t i, int precision_bf16, int64_t jac_for, CenterTerms& ct,
                  CenterTables* tab = nullptr) {
  const int D = m.D, H = m.H, nR = m.nR, nA = m.nA, kR = m.kR, kA = m.kA, L3 = m.L3;
  std::vector<int32_t> nb;
  neighbors_of(g, n, x, box, m.rcR, i, nb);
  ct.pairs.clear();
  for (int32_t j : nb) {
    PairGeom pg;
    pg.j = j;
    pair_vec(x, box, i, j, pg.d);
    pg.r = std::sqrt(r2_of(pg.d));
    for (int c = 0; c < 3; ++c) pg.u[c] = pg.d[c] / pg.r;
    ct.pairs.push_back(pg);
  }
  const int np = (int)ct.pairs.size();
  const int ti = type[i];
  // ZBL: half of each pair's repulsion belongs to U_i.
  double Uz = 0.0;
  ct.zd.assign(np, 0.0);
  for (int p = 0; p < np; ++p) {
    double e, de;
    zbl_pair(m, ti, type[ct.pairs[p].j], ct.pairs[p].r, e, de);
    Uz += 0.5 * e;
    ct.zd[p] = 0.5 * de;
  }
  // Radial functions g_n and derivatives for both cutoffs.
  std::vector<double> gR(np * nR), dgR(np * nR), gA(np * nA, 0.0), dgA(np * nA, 0.0);
  std::vector<char> isA(np, 0);
  std::vector<double> f(std::max(kR, kA)), df(std::max(kR, kA));
  if (tab) {
    tab->fR.assign((size_t)np * kR, 0.0);
    tab->dfR.assign((size_t)np * kR, 0.0);
    tab->fA.assign((size_t)np * kA, 0.0);
    tab->dfA.assign((size_t)np * kA, 0.0);
  }
  for (int p = 0; p < np; ++p) {
    const int tj = type[ct.pairs[p].j];
    const double r = ct.pairs[p].r;
    radial_basis(r, m.rcR, kR, f.data(), df.data());
    if (tab)
      for (int k = 0; k < kR; ++k) {
        tab->fR[(size_t)p * kR + k] = f[k];
        tab->dfR[(size_t)p * kR + k] = df[k];
      }
    const double* c = m.cR + ((int64_t)ti * m.T + tj) * nR * kR;
    for (int a = 0; a < nR; ++a) {
      double s = 0, ds = 0;
      for (int k = 0; k < kR; ++k) { s += c[a * kR + k] * f[k]; ds += c[a * kR + k] * df[k]; }
      gR[p * nR + a] = s;
      dgR[p * nR + a] = ds;
    }
    if (r < m.rcA) {
      isA[p] = 1;
      radial_basis(r, m.rcA, kA, f.data(), df.data());
      if (tab)
        for (int k = 0; k < kA; ++k) {
          tab->fA[(size_t)p * kA + k] = f[k];
          tab->dfA[(size_t)p * kA + k] = df[k];
        }
      const double* ca = m.cA + ((int64_t)ti * m.T + tj) * nA * kA;
      for (int a = 0; a < nA; ++a) {
        double s = 0, ds = 0;
        for (int k = 0; k < kA; ++k) { s += ca[a * kA + k] * f[k]; ds += ca[a * kA + k] * df[k]; }
        gA[p * nA + a] = s;
        dgA[p * nA + a] = ds;
      }
    }
  }
  ct.q.assign(D, 0.0);
  // Radial descriptors.
  for (int p = 0; p < np; ++p)
    for (int a = 0; a < nR; ++a) ct.q[a] += gR[p * nR + a];
  // Angular descriptors via the Legendre double sum over angular neighbours.
  std::vector<int> ang;
  for (int p = 0; p < np; ++p)
    if (isA[p]) ang.push_back(p);
  const int na = (int)ang.size();
  std::vector<double> P(L3 + 1), dP(L3 + 1);
  std::vector<double> cosjk(na * na), Pjk(na * na * (L3 + 1)), dPjk(na * na * (L3 + 1));
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b) {
      const double* ua = ct.pairs[ang[a]].u;
      const double* ub = ct.pairs[ang[b]].u;
      double c = ua[0] * ub[0] + ua[1] * ub[1] + ua[2] * ub[2];
      if (a == b) c = 1.0;
      cosjk[a * na + b] = c;
      legendre(c, L3, P.data(), dP.data());
      for (int l = 0; l <= L3; ++l) {
        Pjk[(a * na + b) * (L3 + 1) + l] = P[l];
        dPjk[(a * na + b) * (L3 + 1) + l] = dP[l];
      }
    }
  for (int l = 1; l <= L3; ++l)
    for (int nn = 0; nn < nA; ++nn) {
      double s = 0;
      for (int a = 0; a < na; ++a)
        for (int b = 0; b < na; ++b)
          s += gA[ang[a] * nA + nn] * gA[ang[b] * nA + nn] * Pjk[(a * na + b) * (L3 + 1) + l];
      ct.q[nR + (l - 1) * nA + nn] = s;
    }
  // Four-body: S_n = sum_j g_n (u u^T - I/3), q4 = tr(S^3).
  std::vector<double> S(nA * 9, 0.0);
  if (m.L4 == 2) {
    for (int a = 0; a < na; ++a) {
      const double* u = ct.pairs[ang[a]].u;
      for (int nn = 0; nn < nA; ++nn) {
        const double gv = gA[ang[a] * nA + nn];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c)
            S[nn * 9 + r * 3 + c] += gv * (u[r] * u[c] - (r == c ? 1.0 / 3.0 : 0.0));
      }
    }
    for (int nn = 0; nn < nA; ++nn) {
      const double* Sm = &S[nn * 9];
      double S2[9], tr = 0;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += Sm[r * 3 + k] * Sm[k * 3 + c];
          S2[r * 3 + c] = s;
        }
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) tr += S2[r * 3 + k] * Sm[k * 3 + r];
      ct.q[nR + L3 * nA + nn] = tr;
    }
  }
  if (tab) {
    tab->gA = gA;
    tab->dgA = dgA;
    tab->ang = ang;
    tab->cosjk = cosjk;
    tab->Pjk = Pjk;
    tab->dPjk = dPjk;
    tab->S = S;
  }
  network(m, ct.q.data(), precision_bf16, ct.U, ct.Fp, ct.h);
  ct.U += Uz;
  if (jac_for == -2) return;
  // Jacobian dq_nu / d r_ij for the requested radial neighbours.
  ct.J.assign((size_t)np * D * 3, 0.0);
  for (int p = 0; p < np; ++p) {
    if (jac_for >= 0 && ct.pairs[p].j != jac_for) continue;
    const double* u = ct.pairs[p].u;
    for (int a = 0; a < nR; ++a)
      for (int c = 0; c < 3; ++c) ct.J[((size_t)p * D + a) * 3 + c] = dgR[p * nR + a] * u[c];
  }
  for (int a = 0; a < na; ++a) {
    const int p = ang[a];
    if (jac_for >= 0 && ct.pairs[p].j != jac_for) continue;
    const double* uj = ct.pairs[p].u;
    const double rj = ct.pairs[p].r;
    for (int l = 1; l <= L3; ++l)
      for (int nn = 0; nn < nA; ++nn) {
        double acc[3] = {0, 0, 0};
        const double gj = gA[p * nA + nn], dgj = dgA[p * nA + nn];
        for (int b = 0; b < na; ++b) {
          const double gk = gA[ang[b] * nA + nn];
          const double c = cosjk[a * na + b];
          const double Pl = Pjk[(a * na + b) * (L3 + 1) + l];
          const double dPl = dPjk[(a * na + b) * (L3 + 1) + l];
          const double* uk = ct.pairs[ang[b]].u;
          for (int cc = 0; cc < 3; ++cc)
            acc[cc] += gk * (dgj * Pl * uj[cc] + gj * dPl * (uk[cc] - c * uj[cc]) / rj);
        }
        for (int cc = 0; cc < 3; ++cc)
          ct.J[((size_t)p * D + nR + (l - 1) * nA + nn) * 3 + cc] = 2.0 * acc[cc];
      }
    if (m.L4 == 2) {
      for (int nn = 0; nn < nA; ++nn) {
        const double* Sm = &S[nn * 9];
        double S2[9];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += Sm[r * 3 + k] * Sm[k * 3 + c];
            S2[r * 3 + c] = s;
          }
        const double gj = gA[p * nA + nn], dgj = dgA[p * nA + nn];
        for (int cc = 0; cc < 3; ++cc) {
          // dS_ab / d(r_j)_cc
          double tr = 0;
          for (int ai = 0; ai < 3; ++ai)
            for (int bi = 0; bi < 3; ++bi) {
              const double Mab = uj[ai] * uj[bi] - (ai == bi ? 1.0 / 3.0 : 0.0);
              const double duu = ((ai == cc ? 1.0 : 0.0) - uj[ai] * uj[cc]) * uj[bi] / rj +
                                 uj[ai] * ((bi == cc ? 1.0 : 0.0) - uj[bi] * uj[cc]) / rj;
              const double dS = dgj * uj[cc] * Mab + gj * duu;
              tr += S2[bi * 3 + ai] * dS;
            }
          ct.J[((size_t)p * D + nR + L3 * nA + nn) * 3 + cc] = 3.0 * tr;
        }
      }
    }
  }
}

// dU_i / d r_ij = sum_nu Fp_nu dq_nu/dr_ij (+ the ZBL half pair term along u) for pair p of center ct.
void pair_force(const CenterTerms& ct, int D, int p, double* out) {
  out[0] = out[1] = out[2] = 0.0;
  for (int v = 0; v < D; ++v)
    for (int c = 0; c < 3; ++c) out[c] += ct.Fp[v] * ct.J[((size_t)p * D + v) * 3 + c];
  for (int c = 0; c < 3; ++c) out[c] += ct.zd[p] * ct.pairs[p].u[c];
}

int find_pair(const CenterTerms& ct, int32_t j) {
  int lo = 0, hi = (int)ct.pairs.size() - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (ct.pairs[mid].j == j) return mid;
    if (ct.pairs[mid].j < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int nthreads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Per-center record kept for force assembly: neighbour ids and dU_i/dr_ij.
struct CenterForces {
  double U = 0;
  std::vector<int32_t> j;
  std::vector<double> d;  // [npairs][3]
};

int find_in(const CenterForces& cf, int32_t j) {
  const auto it = std::lower_bound(cf.j.begin(), cf.j.end(), j);
  if (it == cf.j.end() || *it != j) return -1;
  return (int)(it - cf.j.begin());
}

// Full evaluation of all atoms: per-atom U, forces F_i = sum_j [dU_i/dr_ij - dU_j/dr_ji],
// total energy and virial W_ab = -sum_i sum_j (r_ij)_a (dU_i/dr_ij)_b.
int evaluate_all(const Model& m, int64_t n, const double* x, const int32_t* type, const double* box,
                 int bf16, double* U, double* F, double* E, double* W) {
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  CellGrid g;
  const bool use_grid = n > 256;
  if (use_grid) g.build(n, x, box, m.rcR);
  std::vector<CenterForces> rec(n);
  std::vector<double> Wpart((size_t)n * 9, 0.0);
#pragma omp parallel
  {
    CenterTerms ct;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      center_terms(m, use_grid ? &g : nullptr, n, x, type, box, i, bf16, -1, ct);
      const int np = (int)ct.pairs.size();
      rec[i].U = ct.U;
      rec[i].j.resize(np);
      rec[i].d.resize((size_t)np * 3);
      double w[9] = {0};
      for (int p = 0; p < np; ++p) {
        double f[3];
        pair_force(ct, m.D, p, f);
        rec[i].j[p] = ct.pairs[p].j;
        for (int c = 0; c < 3; ++c) rec[i].d[3 * p + c] = f[c];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) w[a * 3 + b] -= ct.pairs[p].d[a] * f[b];
      }
      for (int k = 0; k < 9; ++k) Wpart[(size_t)i * 9 + k] = w[k];
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double fi[3] = {0, 0, 0};
    const CenterForces& ci = rec[i];
    for (size_t p = 0; p < ci.j.size(); ++p) {
      const CenterForces& cj = rec[ci.j[p]];
      const int q = find_in(cj, (int32_t)i);
      for (int c = 0; c < 3; ++c) fi[c] += ci.d[3 * p + c] - (q >= 0 ? cj.d[3 * q + c] : 0.0);
    }
    if (F) for (int c = 0; c < 3; ++c) F[3 * i + c] = fi[c];
    if (U) U[i] = ci.U;
  }
  double e = 0, w[9] = {0};
  for (int64_t i = 0; i < n; ++i) {
    e += rec[i].U;
    for (int k = 0; k < 9; ++k) w[k] += Wpart[(size_t)i * 9 + k];
  }
  if (E) *E = e;
  if (W) for (int k = 0; k < 9; ++k) W[k] = w[k];
  return OK;
}

}  // namespace

extern "C" {

int orc_num_threads() { return nthreads(); }

// Number of OpenMP threads for the following calls (n >= 1), to time the oracle on
// one core and on all of them.
int orc_set_num_threads(int32_t n) {
  if (n < 1) return ERR_ARG;
#ifdef _OPENMP
  omp_set_num_threads(n);
#endif
  return OK;
}

int orc_n_params(const int32_t* ip, int64_t* n_params, int32_t* n_desc) {
  if (!ip) return ERR_ARG;
  Model m;
  std::vector<double> dummy(1);
  const double dp[2] = {6.0, 5.0};
  // Compute the size by parsing with a trial count.
  const int64_t T = ip[0], nR = ip[1] + 1, nA = ip[2] + 1, kR = ip[3] + 1, kA = ip[4] + 1;
  const int64_t D = nR + nA * ip[5] + (ip[6] == 2 ? nA : 0);
  const int64_t H = ip[7];
  const int64_t np = T * T * nR * kR + T * T * nA * kA + D + H * D + H + H + 1;
  (void)m; (void)dp;
  if (n_params) *n_params = np;
  if (n_desc) *n_desc = (int32_t)D;
  return OK;
}

// Neighbour lists with r2 < cut^2, ascending ids. counts[n]; idx[n][cap].
// Returns ERR_CAP if any count exceeds cap (counts still hold the true counts).
int orc_neighbors(int64_t n, const double* x, const double* box, double cut, int brute,
                  int64_t* counts, int32_t* idx, int32_t cap) {
  if (!x || !box || !counts || n < 1 || !(cut > 0)) return ERR_ARG;
  if (!box_ok(box, cut)) return ERR_BOX;
  CellGrid g;
  if (!brute) g.build(n, x, box, cut);
  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : overflow)
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int32_t> nb;
    neighbors_of(brute ? nullptr : &g, n, x, box, cut, i, nb);
    counts[i] = (int64_t)nb.size();
    if ((int64_t)nb.size() > cap) overflow = 1;
    if (idx)
      for (int64_t k = 0; k < (int64_t)nb.size() && k < cap; ++k) idx[i * cap + k] = nb[k];
  }
  return overflow ? ERR_CAP : OK;
}

// Radial basis f_k(r) and derivatives (K functions) at one distance.
int orc_radial_basis(double r, double rc, int32_t K, double* f, double* df) {
  if (!f || !df || K < 1) return ERR_ARG;
  radial_basis(r, rc, K, f, df);
  return OK;
}

int orc_legendre(double c, int32_t L, double* P, double* dP) {
  if (!P || !dP || L < 1) return ERR_ARG;
  legendre(c, L, P, dP);
  return OK;
}

// Real spherical harmonics of degree l at unit vector u (2l+1 values, m = -l..l).
int orc_sph_harm(int32_t l, const double* u, double* Y) {
  if (!u || !Y || l < 0) return ERR_ARG;
  real_sph_harm(l, u, Y);
  return OK;
}

double orc_round_bf16(double v) { return round_bf16(v); }

// The network alone on a given descriptor vector q [D]: U and Fp = dU/dq [D].
int orc_network(const int32_t* ip, const double* dp, const double* params, int64_t n_params, const double* q,
                int32_t bf16, double* U, double* Fp) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!q || !U || !Fp) return ERR_ARG;
  std::vector<double> fp, h;
  network(m, q, bf16, *U, fp, h);
  for (int v = 0; v < m.D; ++v) Fp[v] = fp[v];
  return OK;
}

// Descriptors q[ncent][D] of the listed centers. path 0: Legendre double sum (the
// path the oracle's forces use); path 1: spherical-harmonic sums s_nlm contracted
// over m, computed independently from the real harmonics above.
int orc_descriptors(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                    int64_t n, const double* x, const int32_t* type, const double* box,
                    int64_t ncent, const int64_t* centers, int32_t path, double* q) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  CellGrid g;
  const bool use_grid = n > 256;
  if (use_grid) g.build(n, x, box, m.rcR);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < ncent; ++c) {
    const int64_t i = centers ? centers[c] : c;
    CenterTerms ct;
    center_terms(m, use_grid ? &g : nullptr, n, x, type, box, i, 0, -2, ct);
    if (path == 1) {
      // Replace the angular block by the spherical-harmonic form.
      const int ti = type[i];
      std::vector<double> s((size_t)m.nA * (m.L3 + 1) * (2 * m.L3 + 1), 0.0);
      std::vector<double> f(m.kA), df(m.kA), Y(2 * m.L3 + 1);
      std::vector<double> sS(m.nA * 9, 0.0);
      for (const PairGeom& pg : ct.pairs) {
        if (!(pg.r < m.rcA)) continue;
        radial_basis(pg.r, m.rcA, m.kA, f.data(), df.data());
        const double* ca = m.cA + ((int64_t)ti * m.T + type[pg.j]) * m.nA * m.kA;
        for (int nn = 0; nn < m.nA; ++nn) {
          double gv = 0;
          for (int k = 0; k < m.kA; ++k) gv += ca[nn * m.kA + k] * f[k];
          for (int l = 1; l <= m.L3; ++l) {
            real_sph_harm(l, pg.u, Y.data());
            for (int mm = 0; mm < 2 * l + 1; ++mm)
              s[((size_t)nn * (m.L3 + 1) + l) * (2 * m.L3 + 1) + mm] += gv * Y[mm];
          }
        }
      }
      for (int l = 1; l <= m.L3; ++l)
        for (int nn = 0; nn < m.nA; ++nn) {
          double acc = 0;
          for (int mm = 0; mm < 2 * l + 1; ++mm) {
            const double v = s[((size_t)nn * (m.L3 + 1) + l) * (2 * m.L3 + 1) + mm];
            acc += v * v;
          }
          ct.q[m.nR + (l - 1) * m.nA + nn] = 4.0 * kPi / (2.0 * l + 1.0) * acc;
        }
    }
    for (int v = 0; v < m.D; ++v) q[c * m.D + v] = ct.q[v];
  }
  return OK;
}

// Energy, per-atom energies, forces and virial of the whole system.
// bf16 != 0 rounds the network's matrix operands to bfloat16 (FP64 accumulation).
int orc_evaluate(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                 int64_t n, const double* x, const int32_t* type, const double* box, int32_t bf16,
                 double* energy, double* virial9, double* U, double* F) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!x || !type || !box || n < 1) return ERR_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] >= m.T) return ERR_ARG;
  return evaluate_all(m, n, x, type, box, bf16, U, F, energy, virial9);
}

// Per-atom energies and forces of sampled atoms only (ascending or any order).
// Evaluates the sampled atoms and all their radial neighbours.
int orc_evaluate_sampled(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                         int64_t n, const double* x, const int32_t* type, const double* box,
                         int32_t bf16, int64_t nsel, const int64_t* sel, double* U_sel, double* F_sel) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!x || !type || !box || !sel || nsel < 1) return ERR_ARG;
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  CellGrid g;
  g.build(n, x, box, m.rcR);
  std::vector<CenterTerms> own(nsel);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t s = 0; s < nsel; ++s) {
    const int64_t i = sel[s];
    center_terms(m, &g, n, x, type, box, i, bf16, -1, own[s]);
    double fi[3] = {0, 0, 0};
    for (int p = 0; p < (int)own[s].pairs.size(); ++p) {
      double f[3];
      pair_force(own[s], m.D, p, f);
      CenterTerms cj;
      center_terms(m, &g, n, x, type, box, own[s].pairs[p].j, bf16, i, cj);
      const int q = find_pair(cj, (int32_t)i);
      double fr[3] = {0, 0, 0};
      if (q >= 0) pair_force(cj, m.D, q, fr);
      for (int c = 0; c < 3; ++c) fi[c] += f[c] - fr[c];
    }
    if (U_sel) U_sel[s] = own[s].U;
    if (F_sel) for (int c = 0; c < 3; ++c) F_sel[3 * s + c] = fi[c];
  }
  return OK;
}

// Per-atom energies only (descriptor + network), for sampled or all atoms.
int orc_energies(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                 int64_t n, const double* x, const int32_t* type, const double* box, int32_t bf16,
                 int64_t ncent, const int64_t* centers, double* U, double* Fp, double* q) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  CellGrid g;
  const bool use_grid = n > 256;
  if (use_grid) g.build(n, x, box, m.rcR);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < ncent; ++c) {
    const int64_t i = centers ? centers[c] : c;
    CenterTerms ct;
    center_terms(m, use_grid ? &g : nullptr, n, x, type, box, i, bf16, -2, ct);
    if (U) U[c] = ct.U;
    if (Fp) for (int v = 0; v < m.D; ++v) Fp[c * m.D + v] = ct.Fp[v];
    if (q) for (int v = 0; v < m.D; ++v) q[c * m.D + v] = ct.q[v];
  }
  return OK;
}

// The per-center work of one force evaluation (descriptor, network and every
// pair derivative dU_i/dr_ij) for ncent consecutive centers starting at first.
// Returns the sum of |dU_i/dr_ij| components as a checksum.
int orc_center_work(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                    int64_t n, const double* x, const int32_t* type, const double* box,
                    int64_t first, int64_t ncent, double* checksum) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  if (first < 0 || first + ncent > n) return ERR_ARG;
  CellGrid g;
  g.build(n, x, box, m.rcR);
  double total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t c = 0; c < ncent; ++c) {
    CenterTerms ct;
    center_terms(m, &g, n, x, type, box, first + c, 0, -1, ct);
    for (int p = 0; p < (int)ct.pairs.size(); ++p) {
      double f[3];
      pair_force(ct, m.D, p, f);
      total += std::fabs(f[0]) + std::fabs(f[1]) + std::fabs(f[2]);
    }
  }
  if (checksum) *checksum = total;
  return OK;
}

// Velocity Verlet in FP64: n_steps steps of dt (fs). x, v updated in place.
// thermo[(s)][4] = {potential energy, kinetic energy, temperature, pressure} after
// each step s (including step 0 = initial state at index 0, so n_steps+1 rows).
int orc_velocity_verlet(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                        int64_t n, double* x, double* v, const int32_t* type, const double* masses,
                        const double* box, double dt, int64_t n_steps, double* thermo) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  std::vector<double> F(3 * n);
  double E = 0, W[9];
  st = evaluate_all(m, n, x, type, box, 0, nullptr, F.data(), &E, W);
  if (st) return st;
  const double V = box[0] * box[1] * box[2];
  auto thermo_row = [&](int64_t s) {
    if (!thermo) return;
    double ke = 0;
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) ke += 0.5 * masses[type[i]] * kXi * v[3 * i + c] * v[3 * i + c];
    const double T = 2.0 * ke / ((3.0 * n - 3.0) * kBoltzmann);
    const double Pr = (2.0 * ke + (W[0] + W[4] + W[8])) / (3.0 * V);
    thermo[4 * s + 0] = E;
    thermo[4 * s + 1] = ke;
    thermo[4 * s + 2] = T;
    thermo[4 * s + 3] = Pr;
  };
  thermo_row(0);
  for (int64_t s = 1; s <= n_steps; ++s) {
    for (int64_t i = 0; i < n; ++i) {
      const double inv = 1.0 / (masses[type[i]] * kXi);
      for (int c = 0; c < 3; ++c) {
        v[3 * i + c] += 0.5 * dt * F[3 * i + c] * inv;
        x[3 * i + c] += dt * v[3 * i + c];
        if (x[3 * i + c] < 0.0) x[3 * i + c] += box[c];
        else if (x[3 * i + c] >= box[c]) x[3 * i + c] -= box[c];
      }
    }
    st = evaluate_all(m, n, x, type, box, 0, nullptr, F.data(), &E, W);
    if (st) return st;
    for (int64_t i = 0; i < n; ++i) {
      const double inv = 1.0 / (masses[type[i]] * kXi);
      for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * F[3 * i + c] * inv;
    }
    thermo_row(s);
  }
  return OK;
}

// Nose-Hoover chain (NVT) state and its half step, in the explicit reversible
// Trotter form of Martyna, Tuckerman, Tobias and Klein (Mol. Phys. 87, 1117, 1996).
// The chain has M thermostats with positions eta_k and velocities ve_k (1/fs) and
// masses Q_1 = Nf kT0 tau^2, Q_k = kT0 tau^2 (k >= 2), Nf = 3N - 3; the forces on it are
//   G_1 = (2 KE - Nf kT0) / Q_1,  G_k = (Q_{k-1} ve_{k-1}^2 - kT0) / Q_k.
// One half step of length h = dt/2 moves the outermost velocity by G h/2, sweeps the
// chain inwards (each ve_k damped by exp(-ve_{k+1} h/4) before and after its kick
// G_k h/2), scales the particle velocities by exp(-ve_1 h), advances eta_k by ve_k h,
// then sweeps outwards in the mirror order with freshly computed forces.
struct Chain {
  int M = 0;
  double kT = 0, Nf = 0;
  std::vector<double> Q, eta, ve;
  double G(int k, double ke) const {
    if (k == 0) return (2.0 * ke - Nf * kT) / Q[0];
    return (Q[k - 1] * ve[k - 1] * ve[k - 1] - kT) / Q[k];
  }
  // Returns the velocity scale factor; ke is updated to the scaled kinetic energy.
  double half_step(double h, double& ke) {
    const int L = M - 1;
    ve[L] += G(L, ke) * h / 2;
    for (int k = L - 1; k >= 0; --k) {
      const double d = std::exp(-ve[k + 1] * h / 4);
      ve[k] *= d;
      ve[k] += G(k, ke) * h / 2;
      ve[k] *= d;
    }
    const double sc = std::exp(-ve[0] * h);
    ke *= sc * sc;
    for (int k = 0; k < M; ++k) eta[k] += ve[k] * h;
    for (int k = 0; k < L; ++k) {
      const double d = std::exp(-ve[k + 1] * h / 4);
      ve[k] *= d;
      ve[k] += G(k, ke) * h / 2;
      ve[k] *= d;
    }
    ve[L] += G(L, ke) * h / 2;
    return sc;
  }
  // The chain's share of the conserved energy.
  double energy() const {
    double e = Nf * kT * eta[0];
    for (int k = 0; k < M; ++k) e += 0.5 * Q[k] * ve[k] * ve[k];
    for (int k = 1; k < M; ++k) e += kT * eta[k];
    return e;
  }
};

// NVT velocity Verlet: a chain half step, half kick, drift, forces, half kick, a chain
// half step. eta and ve (length M) are the chain state, updated in place.
// thermo[s][5] = {PE, KE, T, P, conserved energy} for s = 0..n_steps.
int orc_nvt(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n, double* x,
            double* v, const int32_t* type, const double* masses, const double* box, double dt, int64_t n_steps,
            double T0, double tau, int32_t M, double* eta, double* ve, double* thermo) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (M < 1 || !(T0 > 0) || !(tau > 0) || !eta || !ve || n < 2) return ERR_ARG;
  Chain ch;
  ch.M = M;
  ch.kT = kBoltzmann * T0;
  ch.Nf = 3.0 * n - 3.0;
  ch.Q.assign(M, ch.kT * tau * tau);
  ch.Q[0] *= ch.Nf;
  ch.eta.assign(eta, eta + M);
  ch.ve.assign(ve, ve + M);
  std::vector<double> F(3 * n);
  double E = 0, W[9];
  st = evaluate_all(m, n, x, type, box, 0, nullptr, F.data(), &E, W);
  if (st) return st;
  const double V = box[0] * box[1] * box[2];
  auto kinetic = [&]() {
    double ke = 0;
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) ke += 0.5 * masses[type[i]] * kXi * v[3 * i + c] * v[3 * i + c];
    return ke;
  };
  auto row = [&](int64_t s) {
    if (!thermo) return;
    const double ke = kinetic();
    thermo[5 * s + 0] = E;
    thermo[5 * s + 1] = ke;
    thermo[5 * s + 2] = 2.0 * ke / (ch.Nf * kBoltzmann);
    thermo[5 * s + 3] = (2.0 * ke + (W[0] + W[4] + W[8])) / (3.0 * V);
    thermo[5 * s + 4] = E + ke + ch.energy();
  };
  auto thermostat = [&]() {
    double ke = kinetic();
    const double sc = ch.half_step(0.5 * dt, ke);
    for (int64_t k = 0; k < 3 * n; ++k) v[k] *= sc;
  };
  row(0);
  for (int64_t s = 1; s <= n_steps; ++s) {
    thermostat();
    for (int64_t i = 0; i < n; ++i) {
      const double inv = 1.0 / (masses[type[i]] * kXi);
      for (int c = 0; c < 3; ++c) {
        v[3 * i + c] += 0.5 * dt * F[3 * i + c] * inv;
        x[3 * i + c] += dt * v[3 * i + c];
        if (x[3 * i + c] < 0.0) x[3 * i + c] += box[c];
        else if (x[3 * i + c] >= box[c]) x[3 * i + c] -= box[c];
      }
    }
    st = evaluate_all(m, n, x, type, box, 0, nullptr, F.data(), &E, W);
    if (st) return st;
    for (int64_t i = 0; i < n; ++i) {
      const double inv = 1.0 / (masses[type[i]] * kXi);
      for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * F[3 * i + c] * inv;
    }
    thermostat();
    row(s);
  }
  for (int k = 0; k < M; ++k) {
    eta[k] = ch.eta[k];
    ve[k] = ch.ve[k];
  }
  return OK;
}

// Multiple-time-step (r-RESPA) integration with a fast surrogate force F_s and a
// slow correction F_full - F_s applied every k inner steps:
//   v += (k dt / 2)(F_full - F_s)/(m xi); k velocity-Verlet steps with F_s;
//   evaluate F_full and F_s at the new positions; v += (k dt / 2)(F_full - F_s)/(m xi).
// err[b][2] = {rms, max} over atoms of |F_full - F_s| at the end of block b.
int orc_mts(const int32_t* ipF, const double* dpF, const double* pF, int64_t npF,
            const int32_t* ipS, const double* dpS, const double* pS, int64_t npS,
            int64_t n, double* x, double* v, const int32_t* type, const double* masses,
            const double* box, double dt, int32_t k, int64_t n_blocks, double* err) {
  Model mf, ms;
  int st = parse_model(ipF, dpF, pF, npF, mf);
  if (st) return st;
  st = parse_model(ipS, dpS, pS, npS, ms);
  if (st) return st;
  if (k < 1) return ERR_ARG;
  std::vector<double> Ff(3 * n), Fs(3 * n);
  double E, W[9];
  if ((st = evaluate_all(mf, n, x, type, box, 0, nullptr, Ff.data(), &E, W))) return st;
  if ((st = evaluate_all(ms, n, x, type, box, 0, nullptr, Fs.data(), &E, W))) return st;
  const double big = k * dt;
  for (int64_t b = 0; b < n_blocks; ++b) {
    for (int64_t i = 0; i < n; ++i) {
      const double inv = 1.0 / (masses[type[i]] * kXi);
      for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * big * (Ff[3 * i + c] - Fs[3 * i + c]) * inv;
    }
    for (int s = 0; s < k; ++s) {
      for (int64_t i = 0; i < n; ++i) {
        const double inv = 1.0 / (masses[type[i]] * kXi);
        for (int c = 0; c < 3; ++c) {
          v[3 * i + c] += 0.5 * dt * Fs[3 * i + c] * inv;
          x[3 * i + c] += dt * v[3 * i + c];
          if (x[3 * i + c] < 0.0) x[3 * i + c] += box[c];
          else if (x[3 * i + c] >= box[c]) x[3 * i + c] -= box[c];
        }
      }
      if ((st = evaluate_all(ms, n, x, type, box, 0, nullptr, Fs.data(), &E, W))) return st;
      for (int64_t i = 0; i < n; ++i) {
        const double inv = 1.0 / (masses[type[i]] * kXi);
        for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * Fs[3 * i + c] * inv;
      }
    }
    if ((st = evaluate_all(mf, n, x, type, box, 0, nullptr, Ff.data(), &E, W))) return st;
    double ss = 0, mx = 0;
    for (int64_t i = 0; i < n; ++i) {
      double e2 = 0;
      for (int c = 0; c < 3; ++c) {
        const double e = Ff[3 * i + c] - Fs[3 * i + c];
        e2 += e * e;
      }
      ss += e2;
      mx = std::max(mx, std::sqrt(e2));
    }
    if (err) { err[2 * b] = std::sqrt(ss / (3.0 * n)); err[2 * b + 1] = mx; }
    for (int64_t i = 0; i < n; ++i) {
      const double inv = 1.0 / (masses[type[i]] * kXi);
      for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * big * (Ff[3 * i + c] - Fs[3 * i + c]) * inv;
    }
  }
  return OK;
}

// Gradient of L = gE * E + sum_i gF_i . F_i with respect to the network parameters
// (W0 [H][D], b0 [H], w1 [H], b1), written to grad in that packed order.
// The descriptor coefficients and the scaler are held fixed.
//   energy part:  dU_i/dw1 = t, dU_i/db1 = -1, dU_i/db0 = -w1 d, dU_i/dW0 = (w1 d) qs^T
//   force part:   sum_i gF_i . F_i = -sum_a Fp_a . v_a, with the descriptor JVP
//                 v_a = sum_j dq_a/dr_aj . (gF_j - gF_a), differentiated in closed form.
int orc_weight_grad(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                    int64_t n, const double* x, const int32_t* type, const double* box,
                    double gE, const double* gF, double* grad) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  const int D = m.D, H = m.H;
  const int64_t G = (int64_t)H * D + 2 * H + 1;
  CellGrid g;
  const bool use_grid = n > 256;
  if (use_grid) g.build(n, x, box, m.rcR);
  const int nt = nthreads();
  std::vector<double> part((size_t)nt * G, 0.0);
#pragma omp parallel
  {
#ifdef _OPENMP
    const int tid = omp_get_thread_num();
#else
    const int tid = 0;
#endif
    double* gacc = &part[(size_t)tid * G];
    CenterTerms ct;
    std::vector<double> qs(D), vs(D), z(H);
#pragma omp for schedule(dynamic, 16)
    for (int64_t a = 0; a < n; ++a) {
      center_terms(m, use_grid ? &g : nullptr, n, x, type, box, a, 0, gF != nullptr ? -1 : -2, ct);
      for (int v = 0; v < D; ++v) qs[v] = ct.q[v] * m.sigma[v];
      // descriptor JVP along gF (in scaled-descriptor space)
      for (int v = 0; v < D; ++v) vs[v] = 0;
      if (gF) {
        for (int p = 0; p < (int)ct.pairs.size(); ++p) {
          const int64_t j = ct.pairs[p].j;
          double w[3];
          for (int c = 0; c < 3; ++c) w[c] = gF[3 * j + c] - gF[3 * a + c];
          for (int v = 0; v < D; ++v) {
            double s = 0;
            for (int c = 0; c < 3; ++c) s += ct.J[((size_t)p * D + v) * 3 + c] * w[c];
            vs[v] += s;
          }
        }
        for (int v = 0; v < D; ++v) vs[v] *= m.sigma[v];
      }
      for (int mu = 0; mu < H; ++mu) {
        double s = 0;
        for (int v = 0; v < D; ++v) s += m.W0[mu * D + v] * vs[v];
        z[mu] = s;
      }
      for (int mu = 0; mu < H; ++mu) {
        const double t = std::tanh(ct.h[mu]);
        const double d = 1.0 - t * t;
        const double w1d = m.w1[mu] * d;
        const double zwtd = 2.0 * z[mu] * m.w1[mu] * t * d;
        // W0
        for (int v = 0; v < D; ++v) {
          const double eg = w1d * qs[v];
          const double fg = w1d * vs[v] - zwtd * qs[v];
          gacc[mu * D + v] += gE * eg - fg;
        }
        // b0
        gacc[(int64_t)H * D + mu] += gE * (-w1d) - zwtd;
        // w1
        gacc[(int64_t)H * D + H + mu] += gE * t - z[mu] * d;
      }
      gacc[(int64_t)H * D + 2 * H] += gE * (-1.0);
    }
  }
  for (int64_t k = 0; k < G; ++k) {
    double s = 0;
    for (int t = 0; t < nt; ++t) s += part[(size_t)t * G + k];
    grad[k] = s;
  }
  return OK;
}

// Gradient of L = gE * E + sum_i gF_i . F_i with respect to every packed
// parameter, in the packed order [cR | cA | sigma | W0 | b0 | w1 | b1]: the
// trainable expansion coefficients c^{t_i t_j}_{nk} of the radial functions
// (Section III.B), the descriptor scaler and the network.
// Each center contributes L_a = gE U_a - Fp_a . v_a, with v_a the descriptor JVP
// along gF as in orc_weight_grad. Its derivative with respect to the descriptor
// is rho_a = gE Fp_a - (d^2 U_a / dq^2) v_a = sigma * (W0^T alpha), and with
// respect to v_a it is -Fp_a = -sigma * (W0^T beta), where alpha = gE w1 d +
// 2 z w1 t d and beta = w1 d. The descriptor and its JVP depend on c only through
// the per-pair radial values g_n(r_aj) = sum_k c_nk f_k(r_aj) and their radial
// derivatives g'_n(r_aj) = sum_k c_nk f'_k(r_aj), so
//   dL/dc^{t_a t}_{nk} = sum over neighbours j of type t of
//                        f_k(r_aj) dL_a/dg_n(r_aj) + f'_k(r_aj) dL_a/dg'_n(r_aj),
// and the partial derivatives with respect to g_n and g'_n are taken term by term
// from the radial sum, the Legendre double sum of q_nl and the four-body trace.
int orc_param_grad(const int32_t* ip, const double* dp, const double* params, int64_t n_params,
                   int64_t n, const double* x, const int32_t* type, const double* box,
                   double gE, const double* gF, double* grad) {
  Model m;
  int st = parse_model(ip, dp, params, n_params, m);
  if (st) return st;
  if (!grad) return ERR_ARG;
  if (!box_ok(box, m.rcR)) return ERR_BOX;
  const int D = m.D, H = m.H, T = m.T, nR = m.nR, nA = m.nA, kR = m.kR, kA = m.kA, L3 = m.L3;
  const int64_t G = n_params;
  const int64_t oA = (int64_t)T * T * nR * kR;       // start of cA
  const int64_t oS = oA + (int64_t)T * T * nA * kA;  // start of sigma
  const int64_t oN = m.off_nn;                         // start of W0
  CellGrid g;
  const bool use_grid = n > 256;
  if (use_grid) g.build(n, x, box, m.rcR);
  const int nt = nthreads();
  std::vector<double> part((size_t)nt * G, 0.0);
#pragma omp parallel
  {
#ifdef _OPENMP
    const int tid = omp_get_thread_num();
#else
    const int tid = 0;
#endif
    double* gacc = &part[(size_t)tid * G];
    CenterTerms ct;
    CenterTables tb;
    std::vector<double> qs(D), v(D), vs(D), z(H), t(H), dd(H), al(H), be(H), rho(D), phi(D);
    std::vector<double> w, uw;
#pragma omp for schedule(dynamic, 16)
    for (int64_t a = 0; a < n; ++a) {
      center_terms(m, use_grid ? &g : nullptr, n, x, type, box, a, 0, gF != nullptr ? -1 : -2, ct, &tb);
      const int np = (int)ct.pairs.size();
      const int ti = type[a];
      // w_p = gF_j - gF_a per pair, u_p . w_p, and the JVP v = sum_p J_p w_p
      w.assign((size_t)np * 3, 0.0);
      uw.assign(np, 0.0);
      for (int k = 0; k < D; ++k) v[k] = 0.0;
      if (gF) {
        for (int p = 0; p < np; ++p) {
          const int64_t j = ct.pairs[p].j;
          for (int c = 0; c < 3; ++c) w[3 * p + c] = gF[3 * j + c] - gF[3 * a + c];
          uw[p] = ct.pairs[p].u[0] * w[3 * p] + ct.pairs[p].u[1] * w[3 * p + 1] + ct.pairs[p].u[2] * w[3 * p + 2];
          for (int k = 0; k < D; ++k)
            for (int c = 0; c < 3; ++c) v[k] += ct.J[((size_t)p * D + k) * 3 + c] * w[3 * p + c];
        }
      }
      // network terms
      for (int k = 0; k < D; ++k) {
        qs[k] = ct.q[k] * m.sigma[k];
        vs[k] = v[k] * m.sigma[k];
      }
      for (int mu = 0; mu < H; ++mu) {
        double s = 0;
        for (int k = 0; k < D; ++k) s += m.W0[mu * D + k] * vs[k];
        z[mu] = s;
        t[mu] = std::tanh(ct.h[mu]);
        dd[mu] = 1.0 - t[mu] * t[mu];
        be[mu] = m.w1[mu] * dd[mu];
        al[mu] = gE * be[mu] + 2.0 * z[mu] * m.w1[mu] * t[mu] * dd[mu];
      }
      for (int k = 0; k < D; ++k) {
        double sa = 0, sb = 0;
        for (int mu = 0; mu < H; ++mu) {
          sa += m.W0[mu * D + k] * al[mu];
          sb += m.W0[mu * D + k] * be[mu];
        }
        rho[k] = m.sigma[k] * sa;
        phi[k] = m.sigma[k] * sb;
        // scaler: dL/dsigma_k = q_k (W0^T alpha)_k - v_k (W0^T beta)_k
        gacc[oS + k] += ct.q[k] * sa - v[k] * sb;
      }
      // network parameters
      for (int mu = 0; mu < H; ++mu) {
        const double zwtd = 2.0 * z[mu] * m.w1[mu] * t[mu] * dd[mu];
        for (int k = 0; k < D; ++k) gacc[oN + mu * D + k] += gE * be[mu] * qs[k] - (be[mu] * vs[k] - zwtd * qs[k]);
        gacc[oN + (int64_t)H * D + mu] += -gE * be[mu] - zwtd;
        gacc[oN + (int64_t)H * D + H + mu] += gE * t[mu] - z[mu] * dd[mu];
      }
      gacc[oN + (int64_t)H * D + 2 * H] += -gE;
      // radial coefficients: q_n = sum_j g_n, v_n = sum_j g'_n (u . w)
      for (int p = 0; p < np; ++p) {
        const int tj = type[ct.pairs[p].j];
        double* gc = gacc + ((int64_t)ti * T + tj) * nR * kR;
        for (int nn = 0; nn < nR; ++nn)
          for (int k = 0; k < kR; ++k)
            gc[nn * kR + k] += rho[nn] * tb.fR[(size_t)p * kR + k] - phi[nn] * tb.dfR[(size_t)p * kR + k] * uw[p];
      }
      // angular coefficients
      const int na = (int)tb.ang.size();
      auto Pt = [&](int aa, int bb, int l) { return tb.Pjk[((size_t)aa * na + bb) * (L3 + 1) + l]; };
      auto dPt = [&](int aa, int bb, int l) { return tb.dPjk[((size_t)aa * na + bb) * (L3 + 1) + l]; };
      for (int aa = 0; aa < na; ++aa) {
        const int p = tb.ang[aa];
        const int tj = type[ct.pairs[p].j];
        const double* ua = ct.pairs[p].u;
        const double ra = ct.pairs[p].r;
        double* gc = gacc + oA + ((int64_t)ti * T + tj) * nA * kA;
        for (int nn = 0; nn < nA; ++nn) {
          double Gg = 0.0, Gp = 0.0;  // dL_a/dg_n(r_a), dL_a/dg'_n(r_a)
          for (int l = 1; l <= L3; ++l) {
            double dq = 0.0, dv = 0.0;
            for (int bb = 0; bb < na; ++bb) {
              const int pb = tb.ang[bb];
              const double gb = tb.gA[(size_t)pb * nA + nn], dgb = tb.dgA[(size_t)pb * nA + nn];
              const double* ub = ct.pairs[pb].u;
              const double* wb = &w[3 * pb];
              const double* wa = &w[3 * p];
              const double c = tb.cosjk[(size_t)aa * na + bb];
              // q_nl = sum_{j,k} g_j g_k P_l(c_jk)
              dq += 2.0 * gb * Pt(aa, bb, l);
              // v_nl = 2 sum_{j,k} g_k [g'_j P_l(c_jk) (u_j.w_j) + g_j P_l'(c_jk) (u_k - c_jk u_j).w_j / r_j]
              // with g_a in the role of g_k ...
              const double ua_wb = ua[0] * wb[0] + ua[1] * wb[1] + ua[2] * wb[2];
              dv += 2.0 * (dgb * Pt(bb, aa, l) * uw[pb] + gb * dPt(bb, aa, l) * (ua_wb - c * uw[pb]) / ct.pairs[pb].r);
              // ... and in the role of g_j
              const double ub_wa = ub[0] * wa[0] + ub[1] * wa[1] + ub[2] * wa[2];
              dv += 2.0 * gb * dPt(aa, bb, l) * (ub_wa - c * uw[p]) / ra;
            }
            const int k = nR + (l - 1) * nA + nn;
            Gg += rho[k] * dq - phi[k] * dv;
            Gp += -phi[k] * dq * uw[p];  // dv_nl/dg'_a = (dq_nl/dg_a) (u_a.w_a)
          }
          if (m.L4 == 2) {
            // q4 = tr(S^3), S = sum_j g_j M_j, M_j = u_j u_j^T - I/3;
            // v4 = 3 tr(S^2 Sd), Sd = sum_j [g'_j (u_j.w_j) M_j + g_j N_j],
            // N_j = sum_c w_jc dM_j/d(r_j)_c = [(w - (u.w) u) u^T + u (w - (u.w) u)^T] / r_j
            auto Mof = [](const double* u, double* M) {
              for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) M[r * 3 + c] = u[r] * u[c] - (r == c ? 1.0 / 3.0 : 0.0);
            };
            auto Nof = [](const double* u, const double* wv, double uwv, double r, double* N) {
              double e[3];
              for (int c = 0; c < 3; ++c) e[c] = wv[c] - uwv * u[c];
              for (int r0 = 0; r0 < 3; ++r0)
                for (int c = 0; c < 3; ++c) N[r0 * 3 + c] = (e[r0] * u[c] + u[r0] * e[c]) / r;
            };
            auto mul = [](const double* A, const double* B, double* C) {
              for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                  double s = 0;
                  for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[k * 3 + c];
                  C[r * 3 + c] = s;
                }
            };
            auto tr = [](const double* A, const double* B) {
              double s = 0;
              for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) s += A[r * 3 + c] * B[c * 3 + r];
              return s;
            };
            const double* Sm = &tb.S[nn * 9];
            double S2[9], Sd[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Ma[9], Na[9], M[9], N[9];
            mul(Sm, Sm, S2);
            for (int bb = 0; bb < na; ++bb) {
              const int pb = tb.ang[bb];
              Mof(ct.pairs[pb].u, M);
              Nof(ct.pairs[pb].u, &w[3 * pb], uw[pb], ct.pairs[pb].r, N);
              const double gb = tb.gA[(size_t)pb * nA + nn], dgb = tb.dgA[(size_t)pb * nA + nn];
              for (int e = 0; e < 9; ++e) Sd[e] += dgb * uw[pb] * M[e] + gb * N[e];
            }
            Mof(ua, Ma);
            Nof(ua, &w[3 * p], uw[p], ra, Na);
            double MS[9], SM[9];
            mul(Ma, Sm, MS);
            mul(Sm, Ma, SM);
            for (int e = 0; e < 9; ++e) MS[e] += SM[e];
            const double dq4 = 3.0 * tr(S2, Ma);
            const double dv4 = 3.0 * tr(MS, Sd) + 3.0 * tr(S2, Na);
            const int k = nR + L3 * nA + nn;
            Gg += rho[k] * dq4 - phi[k] * dv4;
            Gp += -phi[k] * dq4 * uw[p];
          }
          for (int k = 0; k < kA; ++k)
            gc[nn * kA + k] += Gg * tb.fA[(size_t)p * kA + k] + Gp * tb.dfA[(size_t)p * kA + k];
        }
      }
    }
  }
  for (int64_t k = 0; k < G; ++k) {
    double s = 0;
    for (int tt = 0; tt < nt; ++tt) s += part[(size_t)tt * G + k];
    grad[k] = s;
  }
  return OK;
}

// One Adam update of theta in place (t is the 1-based step count).
int orc_adam(int64_t n, double* theta, const double* g, double* m1, double* m2, int64_t t,
             double lr, double beta1, double beta2, double eps) {
  if (!theta || !g || !m1 || !m2 || t < 1) return ERR_ARG;
  const double c1 = 1.0 - std::pow(beta1, (double)t);
  const double c2 = 1.0 - std::pow(beta2, (double)t);
  for (int64_t k = 0; k < n; ++k) {
    m1[k] = beta1 * m1[k] + (1.0 - beta1) * g[k];
    m2[k] = beta2 * m2[k] + (1.0 - beta2) * g[k] * g[k];
    const double mh = m1[k] / c1;
    const double vh = m2[k] / c2;
    theta[k] -= lr * mh / (std::sqrt(vh) + eps);
  }
  return OK;
}

}  // extern "C"
