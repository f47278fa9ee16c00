// Runs every entry point of the FP64 oracle once on small seeded inputs, for a build
// with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure: the CPU
// test suite compiles this file together with nep_oracle.cpp and runs it; any report
// fails the run). It checks only that each call returns OK and that its outputs are
// finite; the values are pinned by the Python test suite.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int orc_n_params(const int32_t* ip, int64_t* n_params, int32_t* n_desc);
int orc_neighbors(int64_t n, const double* x, const double* box, double cut, int brute, int64_t* counts,
                  int32_t* idx, int32_t cap);
int orc_radial_basis(double r, double rc, int32_t K, double* f, double* df);
int orc_legendre(double c, int32_t L, double* P, double* dP);
int orc_sph_harm(int32_t l, const double* u, double* Y);
double orc_round_bf16(double v);
int orc_network(const int32_t* ip, const double* dp, const double* params, int64_t n_params, const double* q,
                int32_t bf16, double* U, double* Fp);
int orc_descriptors(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                    const double* x, const int32_t* type, const double* box, int64_t ncent, const int64_t* centers,
                    int32_t path, double* q);
int orc_evaluate(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                 const double* x, const int32_t* type, const double* box, int32_t bf16, double* energy,
                 double* virial9, double* U, double* F);
int orc_evaluate_sampled(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                         const double* x, const int32_t* type, const double* box, int32_t bf16, int64_t nsel,
                         const int64_t* sel, double* U_sel, double* F_sel);
int orc_energies(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                 const double* x, const int32_t* type, const double* box, int32_t bf16, int64_t ncent,
                 const int64_t* centers, double* U, double* Fp, double* q);
int orc_center_work(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                    const double* x, const int32_t* type, const double* box, int64_t first, int64_t ncent,
                    double* checksum);
int orc_velocity_verlet(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                        double* x, double* v, const int32_t* type, const double* masses, const double* box,
                        double dt, int64_t n_steps, double* thermo);
int orc_nvt(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n, double* x,
            double* v, const int32_t* type, const double* masses, const double* box, double dt, int64_t n_steps,
            double T0, double tau, int32_t M, double* eta, double* ve, double* thermo);
int orc_mts(const int32_t* ipF, const double* dpF, const double* pF, int64_t npF, const int32_t* ipS,
            const double* dpS, const double* pS, int64_t npS, int64_t n, double* x, double* v, const int32_t* type,
            const double* masses, const double* box, double dt, int32_t k, int64_t n_blocks, double* err);
int orc_weight_grad(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                    const double* x, const int32_t* type, const double* box, double gE, const double* gF,
                    double* grad);
int orc_param_grad(const int32_t* ip, const double* dp, const double* params, int64_t n_params, int64_t n,
                   const double* x, const int32_t* type, const double* box, double gE, const double* gF,
                   double* grad);
int orc_adam(int64_t n, double* theta, const double* g, double* m1, double* m2, int64_t t, double lr,
             double beta1, double beta2, double eps);
}

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++failures;
  }
}

bool finite(const std::vector<double>& a) {
  for (double v : a)
    if (!std::isfinite(v)) return false;
  return true;
}

struct Model {
  int32_t ip[8];
  double dp[6];
  std::vector<double> p;
  int32_t D = 0;
};

Model make_model(int T, int L3, int L4, int H, double rcR, double rcA, double zbl, uint32_t seed) {
  Model m;
  const int32_t ip[8] = {T, 4, 4, 8, 8, L3, L4, H};
  for (int k = 0; k < 8; ++k) m.ip[k] = ip[k];
  const double dp[6] = {rcR, rcA, zbl / 2, zbl, 29.0, 79.0};
  for (int k = 0; k < 6; ++k) m.dp[k] = dp[k];
  int64_t np = 0;
  orc_n_params(m.ip, &np, &m.D);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 0.1);
  m.p.resize((size_t)np);
  for (double& v : m.p) v = nd(rng);
  // descriptor scaler: O(1) scaled descriptors
  const int64_t off = (int64_t)T * T * 5 * 9 * 2;
  for (int k = 0; k < m.D; ++k) m.p[off + k] = k < 5 ? 0.3 : 2.0;
  return m;
}

}  // namespace

int main() {
  // 4 x 4 x 4 FCC cells, Gaussian displacements, two species
  const double a = 3.615;
  const int nc = 4;
  const double box[3] = {nc * a, nc * a, nc * a};
  const double basis[4][3] = {{0, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}, {0, 0.5, 0.5}};
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd(0.0, 0.1);
  std::vector<double> x;
  std::vector<int32_t> type;
  for (int ix = 0; ix < nc; ++ix)
    for (int iy = 0; iy < nc; ++iy)
      for (int iz = 0; iz < nc; ++iz)
        for (int b = 0; b < 4; ++b) {
          const double c[3] = {ix + basis[b][0], iy + basis[b][1], iz + basis[b][2]};
          for (int d = 0; d < 3; ++d) {
            double v = c[d] * a + nd(rng);
            v -= box[d] * std::floor(v / box[d]);
            x.push_back(v);
          }
          type.push_back((int32_t)(type.size() % 2));
        }
  const int64_t n = (int64_t)type.size();
  std::vector<int32_t> type0(n, 0);
  std::vector<double> v(3 * n);
  for (double& t : v) t = 0.01 * nd(rng);
  const double masses[2] = {63.546, 196.97};

  // basis functions and harmonics
  {
    std::vector<double> f(9), df(9), P(5), dP(5), Y(9);
    expect(orc_radial_basis(3.0, 6.0, 9, f.data(), df.data()) == 0 && finite(f) && finite(df), "radial_basis");
    expect(orc_legendre(0.3, 4, P.data(), dP.data()) == 0 && finite(P), "legendre");
    const double u[3] = {0.48, 0.6, 0.64};
    expect(orc_sph_harm(4, u, Y.data()) == 0 && finite(Y), "sph_harm");
    expect(std::isfinite(orc_round_bf16(0.1)), "round_bf16");
  }
  // neighbour lists, brute force and cells
  {
    const int cap = 256;
    std::vector<int64_t> cnt(n);
    std::vector<int32_t> idx((size_t)n * cap);
    expect(orc_neighbors(n, x.data(), box, 7.0, 0, cnt.data(), idx.data(), cap) == 0, "neighbors cells");
    expect(orc_neighbors(n, x.data(), box, 7.0, 1, cnt.data(), idx.data(), cap) == 0, "neighbors brute");
  }
  const Model full = make_model(1, 4, 2, 30, 6.0, 5.0, 0.0, 1);
  const Model sur = make_model(1, 2, 0, 8, 5.0, 4.0, 0.0, 2);
  const Model two = make_model(2, 4, 2, 30, 6.0, 5.0, 2.0, 3);  // two species with ZBL
  for (const Model* mp : {&full, &sur, &two}) {
    const Model& m = *mp;
    const std::vector<int32_t>& ty = m.ip[0] == 2 ? type : type0;
    const int64_t np = (int64_t)m.p.size();
    std::vector<double> q(m.D, 0.2), Fp(m.D), U(n), F(3 * n), W(9), E(1);
    double u = 0;
    expect(orc_network(m.ip, m.dp, m.p.data(), np, q.data(), 1, &u, Fp.data()) == 0 && std::isfinite(u), "network");
    for (int bf16 = 0; bf16 < 2; ++bf16) {
      expect(orc_evaluate(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, bf16, E.data(), W.data(), U.data(),
                          F.data()) == 0 && finite(U) && finite(F) && finite(W),
             "evaluate");
    }
    const int64_t sel[3] = {0, 17, n - 1};
    std::vector<double> Us(3), Fs(9);
    expect(orc_evaluate_sampled(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, 0, 3, sel, Us.data(),
                                Fs.data()) == 0 && finite(Fs),
           "evaluate_sampled");
    std::vector<double> qd(3 * (size_t)m.D);
    for (int path = 0; path < 2; ++path)
      expect(orc_descriptors(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, 3, sel, path, qd.data()) ==
                 0 && finite(qd),
             "descriptors");
    std::vector<double> Ue(3), Fpe(3 * (size_t)m.D), qe(3 * (size_t)m.D);
    expect(orc_energies(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, 0, 3, sel, Ue.data(), Fpe.data(),
                        qe.data()) == 0 && finite(Ue),
           "energies");
    double cs = 0;
    expect(orc_center_work(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, 5, 20, &cs) == 0, "center_work");
    std::vector<double> gF(3 * n);
    for (double& t : gF) t = nd(rng);
    std::vector<double> gw(30 * 30 + 61), gp((size_t)np);
    expect(orc_weight_grad(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, 0.7, gF.data(), gw.data()) == 0,
           "weight_grad");
    expect(orc_param_grad(m.ip, m.dp, m.p.data(), np, n, x.data(), ty.data(), box, 0.7, gF.data(), gp.data()) == 0 &&
               finite(gp),
           "param_grad");
    std::vector<double> xs = x, vs = v, th(3 * 4);
    expect(orc_velocity_verlet(m.ip, m.dp, m.p.data(), np, n, xs.data(), vs.data(), ty.data(), masses, box, 1.0, 2,
                               th.data()) == 0 && finite(xs) && finite(th),
           "velocity_verlet");
    std::vector<double> eta(3, 0.0), ve(3, 0.0), thn(3 * 5);
    xs = x;
    vs = v;
    expect(orc_nvt(m.ip, m.dp, m.p.data(), np, n, xs.data(), vs.data(), ty.data(), masses, box, 1.0, 2, 300.0, 50.0,
                   3, eta.data(), ve.data(), thn.data()) == 0 && finite(xs) && finite(eta),
           "nvt");
  }
  {
    std::vector<double> xs = x, vs = v, err(2 * 2);
    expect(orc_mts(full.ip, full.dp, full.p.data(), (int64_t)full.p.size(), sur.ip, sur.dp, sur.p.data(),
                   (int64_t)sur.p.size(), n, xs.data(), vs.data(), type0.data(), masses, box, 1.0, 2, 2,
                   err.data()) == 0 && finite(err) && finite(xs),
           "mts");
  }
  {
    std::vector<double> th(50, 0.5), g(50, 0.1), m1(50, 0.0), m2(50, 0.0);
    for (int t = 1; t <= 3; ++t)
      expect(orc_adam(50, th.data(), g.data(), m1.data(), m2.data(), t, 1e-3, 0.9, 0.999, 1e-8) == 0 && finite(th),
             "adam");
  }
  std::printf("sanitize_check: %s (%lld atoms)\n", failures ? "FAILED" : "ok", (long long)n);
  return failures ? 1 : 0;
}
