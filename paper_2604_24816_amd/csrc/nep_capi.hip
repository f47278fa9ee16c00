// C-ABI entry points and the host runtime of one simulated system: workspace
// layout, model upload, the step driver (velocity Verlet and multiple time
// stepping) and error reporting. All device work is enqueued on the system's
// stream; the library allocates no device memory.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <mutex>

#include "../../include/nep.h"
#include "nep_common.h"

using namespace nep;

// Device scratch of nep_compute_energy_forces_virial_noalloc: the workspace of a system of
// at most this many bytes, in a file-scope array that every GPU running the library holds
// for the life of the process (host code reaches it only through hipGetSymbolAddress).
constexpr int64_t kNoallocScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

struct nep_model {
  nep_hparams hp;
  std::vector<double> params;
  int D = 0;
  int64_t n_params = 0;
};

namespace {

constexpr double kXi = 103.642697;          // eV per (amu A^2 / fs^2)
constexpr double kBoltzmann = 8.617333262e-5;  // eV / K
constexpr int kResults = 32;                // doubles of device scalar results

int64_t count_params(const nep_hparams& hp, int* D_out) {
  const int64_t T = hp.n_types, nR = hp.n_max_radial + 1, nA = hp.n_max_angular + 1;
  const int64_t kR = hp.basis_radial + 1, kA = hp.basis_angular + 1;
  const int64_t D = nR + nA * hp.l_max_3b + (hp.l_max_4b == 2 ? nA : 0);
  const int64_t H = hp.n_hidden;
  if (D_out) *D_out = (int)D;
  return T * T * nR * kR + T * T * nA * kA + D + H * D + H + H + 1;
}

bool hp_valid(const nep_hparams* hp) {
  if (!hp) return false;
  return hp->n_types >= 1 && hp->n_types <= kMaxTypes && hp->n_max_radial >= 0 && hp->n_max_angular >= 0 &&
         hp->basis_radial >= 1 && hp->basis_angular >= 1 && hp->l_max_3b >= 1 && hp->l_max_3b <= 4 &&
         (hp->l_max_4b == 0 || hp->l_max_4b == 2) && hp->n_hidden >= 1 && hp->rc_radial > 0 &&
         hp->rc_angular > 0 && hp->rc_angular <= hp->rc_radial && std::isfinite(hp->rc_radial) &&
         (hp->zbl_rc_outer == 0.0 ||
          (hp->zbl_rc_outer > 0 && hp->zbl_rc_inner >= 0 && hp->zbl_rc_inner < hp->zbl_rc_outer &&
           hp->zbl_rc_outer <= hp->rc_radial && hp->zbl_z[0] > 0 && (hp->n_types < 2 || hp->zbl_z[1] > 0)));
}

// Round an FP64 value to bfloat16 bits, nearest-even, directly from FP64.
uint16_t f64_to_bf16_bits(double v) {
  if (v == 0.0) return std::signbit(v) ? 0x8000u : 0u;
  int e = 0;
  const double mant = std::frexp(v, &e);         // |mant| in [0.5, 1)
  const double r = std::nearbyint(std::ldexp(mant, 8));  // 8 significant bits
  const float f = (float)std::ldexp(r, e - 8);   // exactly representable
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

struct Carver {
  int64_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(int64_t count) {
    off = (off + 255) & ~int64_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * (int64_t)sizeof(T);
    return p;
  }
};

CellGrid make_grid(const double box[3], double cut) {
  CellGrid g;
  g.ncell = 8;
  for (int c = 0; c < 3; ++c) {
    int n = (int)std::floor(box[c] / cut);
    while (n > 1 && box[c] / n < cut * (1.0 + 1e-10)) --n;
    if (n < 1) n = 1;
    g.nc[c] = n;
    g.nb[c] = (n + 1) / 2;
    g.box[c] = box[c];
    g.ncell *= g.nb[c];
  }
  return g;
}

}  // namespace

struct nep_system {
  int device = 0;
  hipStream_t st = nullptr;
  int64_t N = 0;
  double box[3] = {0, 0, 0};
  int capR = 0, capA = 0;
  nep_model model[2];
  bool has_model[2] = {false, false};
  ModelDev mdev[2];
  MassTable mt;
  int n_types = 1;
  int max_ncell = 1;
  CellGrid grid;
  bool have_state = false, have_list = false;
  double list_skin = 0;
  bool force_valid[2] = {false, false};
  int force_prec[2] = {0, 0};
  int64_t step = 0;
  int64_t n_mts_blocks = 0, n_fallback_blocks = 0, n_steps_total = 0;
  int judge_relative = 0;  // nep_set_judge
  int deterministic = 0;   // nep_set_deterministic
  // NVT (nep_set_thermostat): Nose-Hoover chain length (0 = NVE), target and period
  int nvt_M = 0;
  double nvt_T = 0, nvt_tau = 0;
  double* nhc = nullptr;  // device chain state {eta[kMaxChain], v_eta[kMaxChain], scale}
  std::string err;
  // device buffers (inside the caller's workspace)
  double *x, *v, *x_alt, *v_alt, *x_build;
  int32_t *type, *type_alt, *perm, *perm_alt, *cellid, *cell_sorted, *src, *key;
  int32_t *cell_count, *cell_start, *cell_fill, *scan_tmp;
  int32_t *nbr, *cnt, *bp, *nactR, *nactA;
  uint16_t *nbrl, *selfl;
  BinEdges be;
  HaloTables ht;
  ListScratch lsc;
  float *F[2], *U, *G;
  uint4 *pos, *rec;
  float *gF, *vjp, *qs;
  double *partial, *gpart, *res, *staging;
  int32_t* flags;
  float* mparams[2];
  float* mderived[2];     // derived radial tables of each model
  float* tderived;        // the same for a parameter vector of the training calls
  uint16_t* mbf[2];
  double* mparams64[2];
  Model64 m64[2];
  int nblocks = 1;
  // kernel timing with events (off unless nep_profile enables it)
  bool prof = false;
  std::vector<hipEvent_t> pool;
  int pool_next = 0;
  std::vector<int> pending;  // triples (start index, stop index, group)
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t prof_cnt[6] = {0, 0, 0, 0, 0, 0};
};

namespace {

constexpr int kGradMax = 32 * 32 + 2 * 32 + 1;  // equals train_grad_stride()
constexpr int kDerivedMax = 10;                 // channels and basis functions the derived tables hold

// Lays out every buffer; with base == nullptr it only measures.
int64_t layout(nep_system* s, char* base, int64_t N, int capR, int capA, int max_ncell, const int64_t* np,
               const int* HD) {
  Carver c;
  c.base = base;
  auto& S = *s;
  S.x = c.take<double>(3 * N);
  S.v = c.take<double>(3 * N);
  S.x_alt = c.take<double>(3 * N);
  S.v_alt = c.take<double>(3 * N);
  S.x_build = c.take<double>(3 * N);
  S.type = c.take<int32_t>(N);
  S.type_alt = c.take<int32_t>(N);
  S.perm = c.take<int32_t>(N);
  S.perm_alt = c.take<int32_t>(N);
  S.cellid = c.take<int32_t>(N);
  S.cell_sorted = c.take<int32_t>(N);
  S.src = c.take<int32_t>(N);
  S.key = c.take<int32_t>(N);
  S.cell_count = c.take<int32_t>(max_ncell);
  S.cell_start = c.take<int32_t>(max_ncell + 1);
  S.cell_fill = c.take<int32_t>(max_ncell);
  S.scan_tmp = c.take<int32_t>(max_ncell / 1024 + 2);
  S.nbr = c.take<int32_t>((int64_t)(capR + kListPad) * N);
  S.cnt = c.take<int32_t>(N);
  S.nbrl = c.take<uint16_t>((int64_t)capR * N);
  S.selfl = c.take<uint16_t>(N);
  S.lsc.q = c.take<uint4>((int64_t)((capR + 15) / 16) * N * 4);
  S.lsc.l = c.take<uint4>((int64_t)((capR + 15) / 16) * N * 2);
  {
    const int64_t nt = grid_blocks(N);
    S.ht.info = c.take<int32_t>(4 * nt);
    S.ht.start = c.take<int32_t>(nt * kHaloCellsMax);
    S.ht.off = c.take<int32_t>(nt * (kHaloCellsMax + 1));
  }
  S.bp = c.take<int32_t>((int64_t)kMaxBins * N);
  S.nactR = c.take<int32_t>(N);
  S.nactA = c.take<int32_t>(N);
  S.F[0] = c.take<float>(3 * N);
  S.F[1] = c.take<float>(3 * N);
  S.U = c.take<float>(N);
  S.pos = c.take<uint4>(N);
  S.rec = c.take<uint4>(4 * N);
  S.G = c.take<float>(5 * 24 * N);
  S.gF = c.take<float>(3 * N);
  const int nb = grid_blocks(N);
  S.partial = c.take<double>((int64_t)nb * kPartialStride);
  S.gpart = c.take<double>((int64_t)nb * kGradMax);
  S.res = c.take<double>(kResults);
  S.staging = c.take<double>(3 * N);
  S.flags = c.take<int32_t>(FLAG_COUNT);
  S.nhc = c.take<double>(kNhcDoubles);
  // derived radial tables: at most kMaxTypes^2 species pairs of kDerivedMax channels and basis functions
  const int64_t nder = derived_coeff_floats(kMaxTypes, kDerivedMax, kDerivedMax, kDerivedMax, kDerivedMax);
  S.tderived = c.take<float>(nder);
  for (int k = 0; k < 2; ++k) {
    S.mderived[k] = c.take<float>(nder);
    S.mparams[k] = c.take<float>(np[k] > 0 ? np[k] : 1);
    S.mbf[k] = c.take<uint16_t>(HD[k] > 0 ? HD[k] : 1);
    S.mparams64[k] = c.take<double>(np[k] > 0 ? np[k] : 1);
  }
  S.vjp = nullptr;
  S.qs = nullptr;
  S.nblocks = nb;
  return (c.off + 255) & ~int64_t(255);
}

#define HIPCHK(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      s->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
      return NEP_ERR_HIP;                                                       \
    }                                                                           \
  } while (0)

// The same for calls without a system to hold the message.
#define HIPCHK2(call)                                                           \
  do {                                                                          \
    if ((call) != hipSuccess) return NEP_ERR_HIP;                               \
  } while (0)

int fail(nep_system* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

// Upload one model's parameters (FP32 copy + bfloat16 copy of W0) into slot `slot`
// (s->model[slot].hp must hold the model's hyperparameters). Host staging uses fixed-size
// arrays, so an upload allocates nothing.
constexpr int kMaxParams = 4096;   // more than any model of a compiled shape (at most 1,921)
constexpr int kMaxNet = 32 * 32;   // network tiles: D <= 32, H <= 32
int upload_model(nep_system* s, int slot, const nep_model& m) {
  const int T = m.hp.n_types, nR = m.hp.n_max_radial + 1, nA = m.hp.n_max_angular + 1;
  const int kR = m.hp.basis_radial + 1, kA = m.hp.basis_angular + 1, H = m.hp.n_hidden, D = m.D;
  if (nR > kDerivedMax || kR > kDerivedMax || nA > kDerivedMax || kA > kDerivedMax || m.n_params > kMaxParams ||
      H * D > kMaxNet)
    return fail(s, NEP_ERR_UNSUPPORTED, "model shape has no compiled kernel");
  float f[kMaxParams];
  for (int64_t k = 0; k < m.n_params; ++k) f[k] = (float)m.params[k];
  const int64_t offW0 = (int64_t)T * T * nR * kR + (int64_t)T * T * nA * kA + D;
  uint16_t bf[kMaxNet];
  for (int k = 0; k < H * D; ++k) bf[k] = f64_to_bf16_bits(m.params[offW0 + k]);
  HIPCHK(hipMemcpyAsync(s->mparams[slot], f, m.n_params * sizeof(float), hipMemcpyHostToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->mbf[slot], bf, H * D * sizeof(uint16_t), hipMemcpyHostToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->mparams64[slot], m.params.data(), m.n_params * sizeof(double),
                        hipMemcpyHostToDevice, s->st));
  HIPCHK(hipStreamSynchronize(s->st));  // the host staging arrays go out of scope
  ModelDev& d = s->mdev[slot];
  d.T = T;
  d.nR = nR;
  d.kR = kR;
  d.nA = nA;
  d.kA = kA;
  d.L3 = m.hp.l_max_3b;
  d.L4 = m.hp.l_max_4b;
  d.H = H;
  d.D = D;
  d.rcR = (float)m.hp.rc_radial;
  d.rcA = (float)m.hp.rc_angular;
  d.rcR64 = m.hp.rc_radial;
  d.rcA64 = m.hp.rc_angular;
  const float* p = s->mparams[slot];
  d.cR = p;
  d.cA = p + (int64_t)T * T * nR * kR;
  d.sigma = d.cA + (int64_t)T * T * nA * kA;
  d.W0 = d.sigma + D;
  d.b0 = d.W0 + (int64_t)H * D;
  d.w1 = d.b0 + H;
  d.b1 = d.w1 + H;
  d.W0bf = s->mbf[slot];
  d.hR = s->mderived[slot];
  d.hA = s->mderived[slot] + (int64_t)T * T * nR * (2 * kR - 1);
  d.hscratch = s->tderived;
  HIPCHK(launch_derive_coeffs(T, nR, kR, nA, kA, d.cR, d.cA, s->mderived[slot], const_cast<float*>(d.hA), s->st));
  {
    Model64& q = s->m64[slot];
    const double* p64 = s->mparams64[slot];
    q.cR = p64;
    q.cA = q.cR + (int64_t)T * T * nR * kR;
    q.sigma = q.cA + (int64_t)T * T * nA * kA;
    q.W0 = q.sigma + D;
    q.b0 = q.W0 + (int64_t)H * D;
    q.w1 = q.b0 + H;
    q.b1 = m.params[offW0 + (int64_t)H * D + 2 * H];
  }
  // ZBL constants per species pair: k_e Z_i Z_j (k_e = e^2 / 4 pi eps0 in eV A) and
  // 1 / a with the universal screening length a = 0.8854 a_0 / (Z_i^0.23 + Z_j^0.23)
  const double zo = m.hp.zbl_rc_outer;
  d.zbl_o2 = zo > 0 ? zo * zo : 0.0;
  d.zbl_ri = m.hp.zbl_rc_inner;
  d.zbl_ro = zo;
  for (int k = 0; k < kMaxTypes * kMaxTypes; ++k) d.zbl_kzz[k] = d.zbl_ainv[k] = 0.0;
  if (zo > 0)
    for (int a = 0; a < T; ++a)
      for (int c = 0; c < T; ++c) {
        const double za = m.hp.zbl_z[a], zc = m.hp.zbl_z[c];
        d.zbl_kzz[a * T + c] = 14.399645478 * za * zc;
        d.zbl_ainv[a * T + c] = (std::pow(za, 0.23) + std::pow(zc, 0.23)) / (0.8854 * 0.529177210903);
      }
  s->force_valid[slot] = false;
  return NEP_OK;
}

EvalBuffers eval_buffers(nep_system* s, int slot) {
  EvalBuffers b;
  b.N = s->N;
  for (int c = 0; c < 3; ++c) b.box[c] = s->box[c];
  b.x = s->x;
  b.type = s->type;
  b.nbr = s->nbr;
  b.bp = s->bp;
  b.nactR = s->nactR;
  b.nactA = s->nactA;
  b.nbrl = s->nbrl;
  b.selfl = s->selfl;
  b.hinfo = s->ht.info;
  b.hstart = s->ht.start;
  b.hoff = s->ht.off;
  b.U = s->U;
  b.pos = s->pos;
  b.rec = s->rec;
  b.G = s->G;
  b.F = s->F[slot];
  b.partial = s->partial;
  b.flags = s->flags;
  b.flag_r = slot == 0 ? FLAG_BIN_R : FLAG_BIN_R1;
  b.flag_a = slot == 0 ? FLAG_BIN_A : FLAG_BIN_A1;
  b.deterministic = s->deterministic;
  return b;
}

hipEvent_t* prof_take(nep_system* s, int n);
void prof_pair(nep_system* s, hipEvent_t* base, int a, int b, int group);

int do_eval(nep_system* s, int slot, int prec) {
  hipEvent_t* ev = prof_take(s, 3);
  HIPCHK(launch_eval(s->mdev[slot], prec, eval_buffers(s, slot), s->st, ev));
  if (ev) {
    prof_pair(s, ev, 0, 1, slot == 0 ? 0 : 4);
    prof_pair(s, ev, 1, 2, slot == 0 ? 1 : 5);
  }
  s->force_valid[slot] = true;
  s->force_prec[slot] = prec;
  return NEP_OK;
}

// Reduce energy + virial partials into res[base .. base+10).
int reduce_ew(nep_system* s, int base) {
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_ENERGY, 10, s->res + base, s->st));
  return NEP_OK;
}

// Merged, sorted distance-bin edges of the list (see BinEdges): r_c + f_k skin for the
// radial and angular cutoffs of both models, so that each model's evaluation visits
// only the entries it can need; each model's bounds are the first edges at or beyond
// its own cutoffs plus f_k skin. Any subset of edges that keeps the outer one gives
// correct bounds (a missing edge only makes a model visit the entries up to the next
// one), so when the union exceeds kMaxBins edges the least useful are dropped: the
// largest skin fractions first (they serve only late in a rebuild interval), the
// surrogate's before the full model's at equal fraction; the exact cutoffs (f = 0)
// and the outer edge are always kept.
BinEdges make_bin_edges(const nep_hparams* hp0, const nep_hparams* hp1, double skin) {
  struct Edge {
    double r;
    int rank;  // removal order: higher goes first; -1 = never removed
  };
  // fixed-size arrays: at most two models x kFracs fractions x two cutoffs
  constexpr int kCand = 2 * kFracs * 2;
  Edge c[kCand];
  int nc = 0;
  const nep_hparams* hps[2] = {hp0, hp1};
  for (int m = 0; m < (hp1 ? 2 : 1); ++m)
    for (int k = 0; k < kFracs; ++k) {
      const int rank = k == 0 ? -1 : 2 * k + m;  // f_k skin, surrogate (m = 1) first at equal k
      c[nc++] = {hps[m]->rc_angular + (double)bin_frac(k) * skin, rank};
      c[nc++] = {hps[m]->rc_radial + (double)bin_frac(k) * skin, rank};
    }
  // the list cutoff is the full model's largest edge; edges beyond it cannot be used
  const double outer = hp0->rc_radial + (double)bin_frac(kFracs - 1) * skin;
  for (int a = 1; a < nc; ++a)  // insertion sort by radius (stable)
    for (int b = a; b > 0 && c[b].r < c[b - 1].r; --b) std::swap(c[b], c[b - 1]);
  Edge u[kCand];  // distinct edges up to the outer one, each with its most useful rank
  int nu = 0;
  for (int a = 0; a < nc; ++a) {
    const Edge& x = c[a];
    if (x.r > outer) break;
    if (nu > 0 && u[nu - 1].r == x.r) {
      const int ra = u[nu - 1].rank, rb = x.rank;
      u[nu - 1].rank = (ra < 0 || rb < 0) ? -1 : std::min(ra, rb);
    } else {
      u[nu++] = x;
    }
  }
  u[nu - 1].rank = -1;  // the outer edge
  while (nu > kMaxBins) {
    int worst = -1;
    for (int a = 0; a < nu; ++a)
      if (u[a].rank >= 0 && (worst < 0 || u[a].rank > u[worst].rank)) worst = a;
    if (worst < 0) break;  // cannot happen: at most four exact cutoffs and the outer edge
    for (int a = worst; a + 1 < nu; ++a) u[a] = u[a + 1];
    --nu;
  }
  BinEdges be{};
  be.nbins = nu;
  for (int b = 0; b < kMaxBins; ++b) be.e2[b] = b < be.nbins ? u[b].r * u[b].r : INFINITY;
  // index of the first edge >= r (the last edge if none)
  auto first_at_or_above = [&](double r) {
    int b = 0;
    while (b < nu && u[b].r < r) ++b;
    return std::min(nu - 1, b);
  };
  const nep_hparams* hp[2] = {hp0, hp1 ? hp1 : hp0};
  for (int m = 0; m < 2; ++m)
    for (int k = 0; k < kFracs; ++k) {
      be.idxR[m][k] = first_at_or_above(hp[m]->rc_radial + (double)bin_frac(k) * skin);
      be.idxA[m][k] = first_at_or_above(hp[m]->rc_angular + (double)bin_frac(k) * skin);
    }
  return be;
}

int rebuild(nep_system* s, double skin, int force) {
  s->be = make_bin_edges(&s->model[0].hp, s->has_model[1] ? &s->model[1].hp : nullptr, skin);
  const ListOut lists{s->nbr, s->cnt, s->bp, s->nbrl, s->selfl};
  HIPCHK(launch_rebuild(s->N, s->grid, s->be, s->capR, s->capA, s->x, s->v, s->type, s->perm, s->x_alt,
                        s->v_alt, s->type_alt, s->perm_alt, s->x_build, s->cellid, s->cell_sorted, s->src,
                        s->key, s->cell_count, s->cell_start, s->cell_fill, s->scan_tmp, s->pos, lists, s->ht, s->lsc,
                        s->flags, s->st));
  (void)force;
  return NEP_OK;
}

int read_flags(nep_system* s, int32_t* f) {
  HIPCHK(hipMemcpyAsync(f, s->flags, FLAG_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return NEP_OK;
}

int check_flags(nep_system* s) {
  int32_t f[FLAG_COUNT];
  int st = read_flags(s, f);
  if (st) return st;
  if (f[FLAG_OVF_R] > 0 || f[FLAG_OVF_A] > 0) {
    char buf[256];
    snprintf(buf, sizeof buf, "neighbour list overflow: need radial capacity %d (have %d), angular %d (have %d)",
             std::max(f[FLAG_OVF_R], 0), s->capR, std::max(f[FLAG_OVF_A], 0), s->capA);
    s->have_list = false;
    return fail(s, NEP_ERR_NEIGHBOR_OVERFLOW, buf);
  }
  if (f[FLAG_TYPE]) return fail(s, NEP_ERR_TYPE, "atom type out of range");
  if (f[FLAG_NONFINITE]) return fail(s, NEP_ERR_NONFINITE, "non-finite positions or velocities");
  return NEP_OK;
}

int check_model_pair(const nep_model* full, const nep_model* sur) {
  if (!full) return NEP_ERR_ARG;
  if (sur) {
    if (sur->hp.n_types != full->hp.n_types) return NEP_ERR_ARG;
    if (sur->hp.rc_radial > full->hp.rc_radial || sur->hp.rc_angular > full->hp.rc_angular) return NEP_ERR_ARG;
  }
  return NEP_OK;
}

constexpr int kPoolEvents = 1024;

int prof_drain(nep_system* s) {
  if (s->pending.empty()) {
    s->pool_next = 0;
    return NEP_OK;
  }
  HIPCHK(hipStreamSynchronize(s->st));
  for (size_t k = 0; k + 3 <= s->pending.size(); k += 3) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, s->pool[s->pending[k]], s->pool[s->pending[k + 1]]));
    s->prof_ms[s->pending[k + 2]] += ms;
    s->prof_cnt[s->pending[k + 2]] += 1;
  }
  s->pending.clear();
  s->pool_next = 0;
  return NEP_OK;
}

// n consecutive events from the pool (nullptr when profiling is off).
hipEvent_t* prof_take(nep_system* s, int n) {
  if (!s->prof) return nullptr;
  if (s->pool_next + n > (int)s->pool.size())
    if (prof_drain(s) != NEP_OK) return nullptr;
  hipEvent_t* e = &s->pool[s->pool_next];
  s->pool_next += n;
  return e;
}

void prof_pair(nep_system* s, hipEvent_t* base, int a, int b, int group) {
  const int i0 = (int)(base - s->pool.data());
  s->pending.push_back(i0 + a);
  s->pending.push_back(i0 + b);
  s->pending.push_back(group);
}

}  // namespace

// Scratch of the allocation-free call (see nep_compute_energy_forces_virial_noalloc).
namespace {
constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device with
// that device current.
int noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kNoallocDevices) return NEP_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NEP_ERR_HIP;
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return NEP_OK;
}
}  // namespace

extern "C" {

const char* nep_status_string(int status) {
  switch (status) {
    case NEP_OK: return "ok";
    case NEP_ERR_ARG: return "invalid argument";
    case NEP_ERR_BOX_TOO_SMALL: return "box too small for cutoff + skin";
    case NEP_ERR_NEIGHBOR_OVERFLOW: return "neighbour list capacity exceeded";
    case NEP_ERR_TYPE: return "atom type out of range";
    case NEP_ERR_NONFINITE: return "non-finite value";
    case NEP_ERR_HIP: return "HIP runtime error";
    case NEP_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case NEP_ERR_STALE_LIST: return "no valid neighbour list";
    case NEP_ERR_UNSUPPORTED: return "model shape has no compiled kernel";
    case NEP_ERR_TOO_LARGE: return "system needs more than the fixed 64 MiB scratch of the allocation-free call";
    default: return "unknown status";
  }
}

const char* nep_last_error(const nep_system* s) { return s ? s->err.c_str() : "null system"; }

int nep_param_count(const nep_hparams* hp, int64_t* n_params, int32_t* n_desc) {
  if (!hp_valid(hp)) return NEP_ERR_ARG;
  int D = 0;
  const int64_t n = count_params(*hp, &D);
  if (n_params) *n_params = n;
  if (n_desc) *n_desc = D;
  return NEP_OK;
}

int nep_model_create(const nep_hparams* hp, const double* params, int64_t n_params, nep_model** out) {
  if (!out || !params || !hp_valid(hp)) return NEP_ERR_ARG;
  int D = 0;
  const int64_t n = count_params(*hp, &D);
  if (n != n_params) return NEP_ERR_ARG;
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(params[k])) return NEP_ERR_NONFINITE;
  nep_model* m = new (std::nothrow) nep_model;
  if (!m) return NEP_ERR_ARG;
  m->hp = *hp;
  m->params.assign(params, params + n);
  m->D = D;
  m->n_params = n;
  if (D > 32 || hp->n_hidden > 32) {
    delete m;
    return NEP_ERR_UNSUPPORTED;
  }
  *out = m;
  return NEP_OK;
}

void nep_model_destroy(nep_model* m) { delete m; }

static int max_cells(const double box[3], double rc) {
  const CellGrid g = make_grid(box, rc);
  return g.ncell;
}

int nep_system_workspace_bytes(const nep_model* full, const nep_model* sur, int64_t n_atoms, const double box[3],
                               int32_t cap_radial, int32_t cap_angular, int64_t* bytes) {
  if (!bytes || !box || n_atoms < 1 || n_atoms >= kMaxAtoms || cap_radial < 1 || cap_angular < 1 ||
      cap_radial > kMaxCap || cap_angular > kMaxCap)
    return NEP_ERR_ARG;
  if (check_model_pair(full, sur)) return NEP_ERR_ARG;
  nep_system tmp;
  const int64_t np[2] = {full->n_params, sur ? sur->n_params : 0};
  const int HD[2] = {full->hp.n_hidden * full->D, sur ? sur->hp.n_hidden * sur->D : 0};
  *bytes = layout(&tmp, nullptr, n_atoms, cap_radial, cap_angular, max_cells(box, full->hp.rc_radial), np, HD);
  return NEP_OK;
}

int nep_system_create(const nep_model* full, const nep_model* sur, int64_t n_atoms, const double box[3],
                      int32_t cap_radial, int32_t cap_angular, void* workspace, int64_t workspace_bytes,
                      void* hip_stream, nep_system** out) {
  if (!out || !box || n_atoms < 1 || n_atoms >= kMaxAtoms || cap_radial < 1 || cap_angular < 1 ||
      cap_radial > kMaxCap || cap_angular > kMaxCap)
    return NEP_ERR_ARG;
  if (check_model_pair(full, sur)) return NEP_ERR_ARG;
  for (int c = 0; c < 3; ++c)
    if (!(box[c] > 0) || !std::isfinite(box[c])) return NEP_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace & 255)) return NEP_ERR_WORKSPACE;
  nep_system* s = new (std::nothrow) nep_system;
  if (!s) return NEP_ERR_ARG;
  s->N = n_atoms;
  for (int c = 0; c < 3; ++c) s->box[c] = box[c];
  s->capR = cap_radial;
  s->capA = cap_angular;
  s->model[0] = *full;
  s->has_model[0] = true;
  if (sur) {
    s->model[1] = *sur;
    s->has_model[1] = true;
  }
  s->n_types = full->hp.n_types;
  s->max_ncell = max_cells(box, full->hp.rc_radial);
  const int64_t np[2] = {full->n_params, sur ? sur->n_params : 0};
  const int HD[2] = {full->hp.n_hidden * full->D, sur ? sur->hp.n_hidden * sur->D : 0};
  const int64_t need = layout(s, nullptr, n_atoms, cap_radial, cap_angular, s->max_ncell, np, HD);
  if (workspace_bytes < need) {
    delete s;
    return NEP_ERR_WORKSPACE;
  }
  layout(s, (char*)workspace, n_atoms, cap_radial, cap_angular, s->max_ncell, np, HD);
  s->st = (hipStream_t)hip_stream;
  {  // NEP_DETERMINISTIC=1 in the environment: deterministic accumulation from the start
    const char* env = std::getenv("NEP_DETERMINISTIC");
    s->deterministic = (env && env[0] == '1' && env[1] == '\0') ? 1 : 0;
  }
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return NEP_ERR_HIP;
  }
  for (int k = 0; k < 2; ++k) {
    if (!s->has_model[k]) continue;
    const int st = upload_model(s, k, s->model[k]);
    if (st) {
      delete s;
      return st;
    }
    if (!eval_supported(s->mdev[k])) {
      delete s;
      return NEP_ERR_UNSUPPORTED;
    }
  }
  if (launch_zero_i32(s->flags, FLAG_COUNT, s->st) != hipSuccess ||
      launch_zero_i32(s->nbr, (int64_t)(cap_radial + kListPad) * n_atoms, s->st) != hipSuccess) {
    delete s;
    return NEP_ERR_HIP;
  }
  for (int t = 0; t < kMaxTypes; ++t) {
    s->mt.mass[t] = 1.0;
    s->mt.inv_mxi[t] = 1.0 / kXi;
  }
  *out = s;
  return NEP_OK;
}

void nep_system_destroy(nep_system* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
  delete s;
}

int nep_system_set_params(nep_system* s, int32_t slot, const double* params, int64_t n_params) {
  if (!s || slot < 0 || slot > 1 || !s->has_model[slot] || !params) return fail(s, NEP_ERR_ARG, "bad slot or params");
  if (n_params != s->model[slot].n_params) return fail(s, NEP_ERR_ARG, "parameter count mismatch");
  for (int64_t k = 0; k < n_params; ++k)
    if (!std::isfinite(params[k])) return fail(s, NEP_ERR_NONFINITE, "non-finite parameter");
  s->model[slot].params.assign(params, params + n_params);
  return upload_model(s, slot, s->model[slot]);
}

int nep_set_state(nep_system* s, const double* x, const double* v, const int32_t* types, const double* masses,
                  int32_t on_device) {
  if (!s || !x || !types || !masses) return fail(s, NEP_ERR_ARG, "null argument");
  for (int t = 0; t < s->n_types; ++t) {
    if (!(masses[t] > 0) || !std::isfinite(masses[t])) return fail(s, NEP_ERR_ARG, "masses must be positive");
    s->mt.mass[t] = masses[t];
    s->mt.inv_mxi[t] = 1.0 / (masses[t] * kXi);
  }
  const int64_t N = s->N;
  CellGrid g = make_grid(s->box, s->model[0].hp.rc_radial);
  HIPCHK(launch_zero_i32(s->flags, FLAG_COUNT, s->st));
  const double* xd = x;
  const double* vd = v;
  const int32_t* td = types;
  if (!on_device) {
    // stage host arrays through the device buffers that the rebuild overwrites anyway
    HIPCHK(hipMemcpyAsync(s->x_alt, x, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->st));
    xd = s->x_alt;
    if (v) {
      HIPCHK(hipMemcpyAsync(s->v_alt, v, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->st));
      vd = s->v_alt;
    }
    HIPCHK(hipMemcpyAsync(s->type_alt, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s->st));
    td = s->type_alt;
  }
  HIPCHK(launch_state_in(N, xd, vd, td, s->n_types, g, s->x, s->v, s->type, s->perm, s->pos, s->flags, s->st));
  int32_t f[FLAG_COUNT];
  int st = read_flags(s, f);
  if (st) return st;
  if (f[FLAG_TYPE]) return fail(s, NEP_ERR_TYPE, "atom type out of range");
  if (f[FLAG_NONFINITE]) return fail(s, NEP_ERR_NONFINITE, "non-finite position or velocity");
  s->have_state = true;
  s->have_list = false;
  s->force_valid[0] = s->force_valid[1] = false;
  s->step = 0;
  return NEP_OK;
}

int nep_build_neighbors(nep_system* s, double skin) {
  if (!s) return NEP_ERR_ARG;
  if (!s->have_state) return fail(s, NEP_ERR_ARG, "no state set");
  if (!(skin >= 0) || !std::isfinite(skin)) return fail(s, NEP_ERR_ARG, "skin must be >= 0");
  const double cut = s->model[0].hp.rc_radial + skin;
  for (int c = 0; c < 3; ++c)
    if (!(s->box[c] >= 2.0 * cut)) return fail(s, NEP_ERR_BOX_TOO_SMALL, "every box side must be >= 2 (rc + skin)");
  s->grid = make_grid(s->box, cut);
  HIPCHK(launch_zero_i32(s->flags, FLAG_COUNT, s->st));
  HIPCHK(launch_set_flag(s->flags, FLAG_REBUILD, 1, s->st));
  int st = rebuild(s, skin, 1);
  if (st) return st;
  st = check_flags(s);
  if (st) return st;
  s->have_list = true;
  s->list_skin = skin;
  s->force_valid[0] = s->force_valid[1] = false;
  return NEP_OK;
}

int nep_export_neighbors(nep_system* s, int32_t which, int64_t* offsets, int32_t* idx, int64_t cap_total) {
  if (!s || !offsets || !idx || which < 0 || which > 1) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "no list built");
  const int64_t N = s->N;
  const int cap = which == 0 ? s->capR : s->capA;
  // rows of original ids are produced in chunks that fit the staging buffer (3N doubles)
  const int64_t chunk = std::max<int64_t>(1, (3 * N * (int64_t)sizeof(double)) / ((int64_t)cap * 4 + 4));
  int32_t* rows = reinterpret_cast<int32_t*>(s->staging);
  int32_t* rcnt = rows + chunk * cap;
  std::vector<int32_t> cnt(N);
  std::vector<int32_t> all((size_t)N * cap);
  for (int64_t o0 = 0; o0 < N; o0 += chunk) {
    const int64_t o1 = std::min(N, o0 + chunk);
    // the angular list with skin is the prefix of bins up to rc_angular + skin
    const int32_t* cnt_src = which == 0 ? s->cnt : s->bp + (int64_t)s->be.idxA[0][kFracs - 1] * N;
    HIPCHK(launch_export(N, s->perm, s->nbr, cnt_src, cap, o0, o1, rows, rcnt, s->st));
    HIPCHK(hipMemcpyAsync(cnt.data() + o0, rcnt, (o1 - o0) * sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(all.data() + o0 * cap, rows, (size_t)(o1 - o0) * cap * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
  }
  offsets[0] = 0;
  for (int64_t o = 0; o < N; ++o) offsets[o + 1] = offsets[o] + cnt[o];
  if (offsets[N] > cap_total) return fail(s, NEP_ERR_ARG, "cap_total too small");
  for (int64_t o = 0; o < N; ++o)
    std::memcpy(idx + offsets[o], all.data() + o * cap, cnt[o] * sizeof(int32_t));
  return NEP_OK;
}

int nep_compute_energy_forces_virial(nep_system* s, int32_t slot, int32_t precision, double* energy,
                                     double* virial9, double* forces, double* per_atom_energy,
                                     int32_t on_device) {
  if (!s || !energy || !virial9 || slot < 0 || slot > 1 || !s->has_model[slot] || precision < 0 || precision > 2)
    return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  const int64_t N = s->N;
  int st;
  // FP64: per-atom energies and dU/dq in the dU/ds buffer (1 + D <= 60 doubles per
  // atom), forces in the sort scratch x_alt; the FP32 forces of the slot are stale after
  double* U64 = reinterpret_cast<double*>(s->G);
  double* F64 = s->x_alt;
  if (precision == NEP_FP64) {
    HIPCHK(launch_eval64(s->mdev[slot], s->m64[slot], eval_buffers(s, slot), U64, U64 + N, F64, s->st));
    s->force_valid[slot] = false;
  } else if ((st = do_eval(s, slot, precision))) {
    return st;
  }
  if ((st = reduce_ew(s, 0))) return st;
  if (forces) {
    double* dst = on_device ? forces : s->staging;
    if (precision == NEP_FP64) HIPCHK(launch_state_out(N, s->perm, F64, dst, s->st));
    else HIPCHK(launch_forces_out(N, s->perm, s->F[slot], dst, s->st));
    if (!on_device) HIPCHK(hipMemcpyAsync(forces, s->staging, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s->st));
  }
  if (per_atom_energy) {
    double* dst = on_device ? per_atom_energy : s->staging;
    if (precision == NEP_FP64) HIPCHK(launch_scalar_out64(N, s->perm, U64, dst, s->st));
    else HIPCHK(launch_scalar_out(N, s->perm, s->U, dst, s->st));
    if (!on_device)
      HIPCHK(hipMemcpyAsync(per_atom_energy, s->staging, N * sizeof(double), hipMemcpyDeviceToHost, s->st));
  }
  double r[10];
  HIPCHK(hipMemcpyAsync(r, s->res, 10 * sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  *energy = r[0];
  for (int k = 0; k < 9; ++k) virial9[k] = r[1 + k];
  bool finite = std::isfinite(r[0]);
  for (int k = 1; k < 10; ++k) finite = finite && std::isfinite(r[k]);
  if (!finite) return fail(s, NEP_ERR_NONFINITE, "non-finite energy or virial");
  return NEP_OK;
}

namespace {

// Thermo row {step, PE, KE, T, P, err_rms, err_max, fallback} from res[0..10) (E, W).
int thermo_row(nep_system* s, double* row, double err_rms, double err_max, int fallback) {
  HIPCHK(launch_kinetic(s->N, s->v, s->type, s->mt, s->partial, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_KE, 1, s->res + 10, s->st));
  double r[11];
  HIPCHK(hipMemcpyAsync(r, s->res, 11 * sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  const double V = s->box[0] * s->box[1] * s->box[2];
  const double ke = r[10];
  row[0] = (double)s->step;
  row[1] = r[0];
  row[2] = ke;
  row[3] = 2.0 * ke / ((3.0 * s->N - 3.0) * kBoltzmann);
  row[4] = (2.0 * ke + (r[1] + r[5] + r[9])) / (3.0 * V);
  row[5] = err_rms;
  row[6] = err_max;
  row[7] = fallback;
  return NEP_OK;
}

// One velocity-Verlet step with model `slot`. The rebuild flag is set on the device
// for the scheduled steps and raised by the drift kernel when an atom has moved
// more than skin/2 since the last build.
int vv_step(nep_system* s, int slot, int prec, double dt, int rebuild_every, double skin) {
  const int64_t next = s->step + 1;
  const int scheduled = (rebuild_every > 0 && next % rebuild_every == 0) ? 1 : 0;
  hipEvent_t* ev = prof_take(s, 4);
  if (ev) HIPCHK(hipEventRecord(ev[0], s->st));
  HIPCHK(launch_set_flag(s->flags, FLAG_REBUILD, scheduled, s->st));
  HIPCHK(launch_kick_drift(s->N, dt, s->grid, s->F[slot], s->type, s->mt, s->x, s->v, s->pos, s->x_build,
                           0.25 * skin * skin, s->flags, s->partial, s->st));
  HIPCHK(launch_select_bin(s->partial, kick_drift_blocks(s->N), s->flags, skin, s->be, s->st));
  if (ev) HIPCHK(hipEventRecord(ev[1], s->st));
  int st = rebuild(s, skin, 0);
  if (st) return st;
  if (ev) {
    HIPCHK(hipEventRecord(ev[2], s->st));
    prof_pair(s, ev, 0, 1, 3);
    prof_pair(s, ev, 1, 2, 2);
  }
  if ((st = do_eval(s, slot, prec))) return st;
  hipEvent_t* ev2 = prof_take(s, 2);
  if (ev2) HIPCHK(hipEventRecord(ev2[0], s->st));
  HIPCHK(launch_kick(s->N, dt, s->F[slot], s->type, s->mt, s->v, s->st));
  if (ev2) {
    HIPCHK(hipEventRecord(ev2[1], s->st));
    prof_pair(s, ev2, 0, 1, 3);
  }
  s->step = next;
  s->n_steps_total++;
  return NEP_OK;
}

// One Nose-Hoover chain half step (dt/2) on the current velocities.
int nhc_half(nep_system* s, double dt) {
  HIPCHK(launch_kinetic(s->N, s->v, s->type, s->mt, s->partial, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_KE, 1, s->res + 18, s->st));
  HIPCHK(launch_nhc_half(s->N, s->res + 18, s->nhc, s->nvt_M, kBoltzmann * s->nvt_T, s->nvt_tau, 0.5 * dt, s->v,
                         s->st));
  return NEP_OK;
}

// Surrogate force error against the full model: rms per component and max
// |F_full - F_surrogate| over atoms; frms (nullable) = rms per component of F_full.
int force_error(nep_system* s, double* rms, double* mx, double* frms = nullptr) {
  HIPCHK(launch_force_error(s->N, s->F[0], s->F[1], s->partial, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_ERR2, 1, s->res + 12, s->st));
  HIPCHK(launch_max_partials(s->partial, s->nblocks, P_ERRMAX, s->res + 13, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_F2, 1, s->res + 14, s->st));
  double r[3];
  HIPCHK(hipMemcpyAsync(r, s->res + 12, 3 * sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  *rms = std::sqrt(r[0] / (3.0 * s->N));
  *mx = r[1];
  if (frms) *frms = std::sqrt(r[2] / (3.0 * s->N));
  return NEP_OK;
}

}  // namespace

int nep_step(nep_system* s, int64_t n_steps, double dt_fs, int32_t rebuild_every, double skin, int32_t mts_k,
             double fallback_rms, double fallback_max, int32_t precision, double* thermo, int32_t thermo_every,
             int64_t max_rows, int64_t* rows_written) {
  if (!s || n_steps < 0 || !(dt_fs > 0) || rebuild_every < 0 || !(skin >= 0) || mts_k < 0 || precision < 0 ||
      precision > 1)
    return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_state) return fail(s, NEP_ERR_ARG, "no state set");
  if (mts_k > 0 && (!s->has_model[1] || n_steps % mts_k != 0))
    return fail(s, NEP_ERR_ARG, "MTS needs a surrogate model and n_steps divisible by mts_k");
  if (mts_k > 0 && s->nvt_M > 0) return fail(s, NEP_ERR_ARG, "the thermostat runs with plain velocity Verlet only");
  if (thermo && (thermo_every < 1 || max_rows < 1)) return fail(s, NEP_ERR_ARG, "thermo_every and max_rows must be >= 1");
  if (rows_written) *rows_written = 0;
  int st;
  if (!s->have_list || s->list_skin != skin) {
    if ((st = nep_build_neighbors(s, skin))) return st;
  }
  int64_t rows = 0;
  auto want_row = [&](bool last) {
    return thermo && rows < max_rows && (last || (s->step % thermo_every == 0));
  };
  if (mts_k == 0) {
    if (!s->force_valid[0] || s->force_prec[0] != precision)
      if ((st = do_eval(s, 0, precision))) return st;
    for (int64_t k = 0; k < n_steps; ++k) {
      if (s->nvt_M > 0 && (st = nhc_half(s, dt_fs))) return st;
      if ((st = vv_step(s, 0, precision, dt_fs, rebuild_every, skin))) return st;
      if (s->nvt_M > 0 && (st = nhc_half(s, dt_fs))) return st;
      // a list that overflowed at a build (scheduled, or early since the last check)
      // stops the run here rather than after n_steps of truncated lists
      if (rebuild_every > 0 && s->step % rebuild_every == 0 && (st = check_flags(s))) return st;
      if (want_row(k == n_steps - 1)) {
        if ((st = reduce_ew(s, 0))) return st;
        if ((st = thermo_row(s, thermo + 8 * rows, 0.0, 0.0, 0))) return st;
        ++rows;
      }
    }
    s->force_valid[1] = false;
  } else {
    // Multiple time stepping (r-RESPA): fast force = surrogate (slot 1), slow force =
    // full - surrogate applied as impulses every mts_k steps.
    if (!s->force_valid[0] || s->force_prec[0] != precision)
      if ((st = do_eval(s, 0, precision))) return st;
    if ((st = reduce_ew(s, 0))) return st;
    if (!s->force_valid[1] || s->force_prec[1] != precision)
      if ((st = do_eval(s, 1, precision))) return st;
    const double big = mts_k * dt_fs;
    const int64_t nblk = n_steps / mts_k;
    int fallback = 0, clean = 0;
    // thresholds: absolute (eV/A), or multiples of the block's own rms full-model force
    auto over = [&](double rms, double mx, double frms) {
      const double scale = s->judge_relative ? frms : 1.0;
      return rms > fallback_rms * scale || mx > fallback_max * scale;
    };
    for (int64_t b = 0; b < nblk; ++b) {
      double rms = 0, mx = 0, frms = 0;
      if (!fallback) {
        HIPCHK(launch_kick_diff(s->N, 0.5 * big, s->F[0], s->F[1], s->type, s->mt, s->v, s->st));
        for (int k = 0; k < mts_k; ++k)
          if ((st = vv_step(s, 1, precision, dt_fs, rebuild_every, skin))) return st;
        if ((st = do_eval(s, 0, precision))) return st;
        if ((st = reduce_ew(s, 0))) return st;
        if ((st = force_error(s, &rms, &mx, &frms))) return st;
        HIPCHK(launch_kick_diff(s->N, 0.5 * big, s->F[0], s->F[1], s->type, s->mt, s->v, s->st));
        s->n_mts_blocks++;
        if (over(rms, mx, frms)) {
          fallback = 1;
          clean = 0;
        }
      } else {
        for (int k = 0; k < mts_k; ++k)
          if ((st = vv_step(s, 0, precision, dt_fs, rebuild_every, skin))) return st;
        if ((st = reduce_ew(s, 0))) return st;
        if ((st = do_eval(s, 1, precision))) return st;  // shadow surrogate evaluation
        if ((st = force_error(s, &rms, &mx, &frms))) return st;
        s->n_fallback_blocks++;
        if (!over(rms, mx, frms)) {
          if (++clean >= 10) fallback = 0;
        } else {
          clean = 0;
        }
      }
      if (want_row(b == nblk - 1)) {
        if ((st = thermo_row(s, thermo + 8 * rows, rms, mx, fallback))) return st;
        ++rows;
      }
      // the block has synchronised already: stop at the first overflowing build
      if ((st = check_flags(s))) return st;
    }
  }
  if (rows_written) *rows_written = rows;
  if ((st = check_flags(s))) return st;
  HIPCHK(hipStreamSynchronize(s->st));
  return NEP_OK;
}

int nep_set_thermostat(nep_system* s, double temperature, double tau_fs, int32_t chain_length) {
  if (!s || chain_length < 0 || chain_length > kMaxChain) return fail(s, NEP_ERR_ARG, "bad argument");
  if (chain_length > 0 && !(temperature > 0 && tau_fs > 0 && std::isfinite(temperature) && std::isfinite(tau_fs)))
    return fail(s, NEP_ERR_ARG, "temperature and tau must be positive");
  if (s->N < 2) return fail(s, NEP_ERR_ARG, "a thermostat needs at least two atoms");
  s->nvt_M = chain_length;
  s->nvt_T = temperature;
  s->nvt_tau = tau_fs;
  double zero[kNhcDoubles] = {0};
  zero[2 * kMaxChain] = 1.0;
  HIPCHK(hipMemcpyAsync(s->nhc, zero, sizeof(zero), hipMemcpyHostToDevice, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return NEP_OK;
}

int nep_set_thermostat_state(nep_system* s, const double* eta, const double* v_eta) {
  if (!s || !eta || !v_eta) return fail(s, NEP_ERR_ARG, "bad argument");
  if (s->nvt_M < 1) return fail(s, NEP_ERR_ARG, "no thermostat set");
  double h[kNhcDoubles] = {0};
  for (int k = 0; k < s->nvt_M; ++k) {
    if (!std::isfinite(eta[k]) || !std::isfinite(v_eta[k])) return fail(s, NEP_ERR_NONFINITE, "non-finite chain state");
    h[k] = eta[k];
    h[kMaxChain + k] = v_eta[k];
  }
  h[2 * kMaxChain] = 1.0;
  HIPCHK(hipMemcpyAsync(s->nhc, h, sizeof(h), hipMemcpyHostToDevice, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return NEP_OK;
}

int nep_get_thermostat(nep_system* s, double* eta, double* v_eta, double* chain_energy) {
  if (!s) return NEP_ERR_ARG;
  double h[kNhcDoubles];
  HIPCHK(hipMemcpyAsync(h, s->nhc, sizeof(h), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  const int M = s->nvt_M;
  for (int k = 0; k < M; ++k) {
    if (eta) eta[k] = h[k];
    if (v_eta) v_eta[k] = h[kMaxChain + k];
  }
  if (chain_energy) {
    // Nf kT eta_1 + kT sum_{k>=2} eta_k + sum_k Q_k v_k^2 / 2
    const double kT = kBoltzmann * s->nvt_T, Nf = 3.0 * s->N - 3.0, t2 = s->nvt_tau * s->nvt_tau;
    double e = 0.0;
    for (int k = 0; k < M; ++k) {
      const double Q = (k == 0 ? Nf : 1.0) * kT * t2;
      e += (k == 0 ? Nf * kT : kT) * h[k] + 0.5 * Q * h[kMaxChain + k] * h[kMaxChain + k];
    }
    *chain_energy = e;
  }
  return NEP_OK;
}

int nep_set_judge(nep_system* s, int32_t relative) {
  if (!s || relative < 0 || relative > 1) return fail(s, NEP_ERR_ARG, "bad argument");
  s->judge_relative = relative;
  return NEP_OK;
}

int nep_set_deterministic(nep_system* s, int32_t deterministic) {
  if (!s || deterministic < 0 || deterministic > 1) return fail(s, NEP_ERR_ARG, "bad argument");
  s->deterministic = deterministic;
  return NEP_OK;
}

int nep_get_state(nep_system* s, double* x, double* v, int64_t* step, int32_t on_device) {
  if (!s) return NEP_ERR_ARG;
  if (!s->have_state) return fail(s, NEP_ERR_ARG, "no state set");
  const int64_t N = s->N;
  if (x) {
    double* dst = on_device ? x : s->staging;
    HIPCHK(launch_state_out(N, s->perm, s->x, dst, s->st));
    if (!on_device) HIPCHK(hipMemcpyAsync(x, s->staging, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s->st));
  }
  if (v) {
    double* dst = on_device ? v : s->staging;
    HIPCHK(launch_state_out(N, s->perm, s->v, dst, s->st));
    if (!on_device) HIPCHK(hipMemcpyAsync(v, s->staging, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s->st));
  }
  if (step) *step = s->step;
  HIPCHK(hipStreamSynchronize(s->st));
  return NEP_OK;
}

int nep_get_stats(nep_system* s, int64_t* stats4) {
  if (!s || !stats4) return NEP_ERR_ARG;
  int32_t f[FLAG_COUNT];
  int st = read_flags(s, f);
  if (st) return st;
  stats4[0] = f[FLAG_NBUILD];
  stats4[1] = s->n_mts_blocks;
  stats4[2] = s->n_fallback_blocks;
  stats4[3] = s->n_steps_total;
  return NEP_OK;
}

int nep_halo_stats(nep_system* s, int64_t* stats4) {
  if (!s || !stats4) return NEP_ERR_ARG;
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  const int64_t nt = grid_blocks(s->N);
  std::vector<int32_t> info((size_t)(4 * nt));
  HIPCHK(hipMemcpyAsync(info.data(), s->ht.info, 4 * nt * sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  int64_t global = 0, max_atoms = 0, max_cells = 0;
  for (int64_t t = 0; t < nt; ++t) {
    if (info[4 * t + 2] == 0) ++global;
    max_cells = std::max<int64_t>(max_cells, info[4 * t + 0]);
    max_atoms = std::max<int64_t>(max_atoms, info[4 * t + 1]);
  }
  stats4[0] = nt;
  stats4[1] = global;
  stats4[2] = max_atoms;
  stats4[3] = max_cells;
  return NEP_OK;
}

int nep_surrogate_error(nep_system* s, int32_t precision, double* err2) {
  if (!s || !err2 || !s->has_model[1] || precision < 0 || precision > 1) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  int st;
  if ((st = do_eval(s, 0, precision))) return st;
  if ((st = do_eval(s, 1, precision))) return st;
  return force_error(s, &err2[0], &err2[1]);
}

int nep_train_forward(nep_system* s, int32_t slot, const float* theta, double* energy, float* forces) {
  if (!s || !theta || !energy || slot < 0 || slot > 1 || !s->has_model[slot]) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  HIPCHK(launch_train_forward(s->mdev[slot], theta, eval_buffers(s, slot), s->st));
  s->force_valid[slot] = false;
  int st;
  if ((st = reduce_ew(s, 0))) return st;
  if (forces) HIPCHK(launch_scatter_vec_f32(s->N, s->perm, s->F[slot], forces, s->st));
  double r;
  HIPCHK(hipMemcpyAsync(&r, s->res, sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  *energy = r;
  if (!std::isfinite(r)) return fail(s, NEP_ERR_NONFINITE, "non-finite energy");
  return NEP_OK;
}

int nep_train_backward(nep_system* s, int32_t slot, const float* theta, double gE, const float* gF, float* grad,
                       int32_t accumulate) {
  if (!s || !theta || !grad || slot < 0 || slot > 1 || !s->has_model[slot]) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  TrainBuffers t;
  t.e = eval_buffers(s, slot);
  t.theta = theta;
  t.gE = gE;
  t.gF = nullptr;
  if (gF) {
    HIPCHK(launch_gather_vec_f32(s->N, s->perm, gF, s->gF, s->st));
    t.gF = s->gF;
  }
  t.vjp = nullptr;
  t.qs = nullptr;
  t.gpart = s->gpart;
  t.grad = grad;
  t.accumulate = accumulate ? 1 : 0;
  HIPCHK(launch_train_backward(s->mdev[slot], t, s->st));
  s->force_valid[slot] = false;
  return NEP_OK;
}

int nep_train_forward_params(nep_system* s, int32_t slot, const float* params, double* energy, float* forces) {
  if (!s || !params || !energy || slot < 0 || slot > 1 || !s->has_model[slot]) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  HIPCHK(launch_train_forward_params(s->mdev[slot], params, eval_buffers(s, slot), s->st));
  s->force_valid[slot] = false;
  int st;
  if ((st = reduce_ew(s, 0))) return st;
  if (forces) HIPCHK(launch_scatter_vec_f32(s->N, s->perm, s->F[slot], forces, s->st));
  double r;
  HIPCHK(hipMemcpyAsync(&r, s->res, sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  *energy = r;
  if (!std::isfinite(r)) return fail(s, NEP_ERR_NONFINITE, "non-finite energy");
  return NEP_OK;
}

int nep_train_backward_params(nep_system* s, int32_t slot, const float* params, double gE, const float* gF,
                              float* grad, int32_t accumulate) {
  if (!s || !params || !grad || slot < 0 || slot > 1 || !s->has_model[slot]) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  TrainBuffers t;
  t.e = eval_buffers(s, slot);
  t.theta = params;
  t.gE = gE;
  t.gF = nullptr;
  if (gF) {
    HIPCHK(launch_gather_vec_f32(s->N, s->perm, gF, s->gF, s->st));
    t.gF = s->gF;
  }
  t.vjp = nullptr;
  t.qs = nullptr;
  t.gpart = s->gpart;
  t.grad = grad;
  t.accumulate = accumulate ? 1 : 0;
  HIPCHK(launch_train_backward_params(s->mdev[slot], t, s->st));
  s->force_valid[slot] = false;
  return NEP_OK;
}

int nep_train_backward64(nep_system* s, int32_t slot, double gE, const double* gF, double* grad) {
  if (!s || !grad || slot < 0 || slot > 1 || !s->has_model[slot]) return fail(s, NEP_ERR_ARG, "bad argument");
  if (!s->have_list) return fail(s, NEP_ERR_STALE_LIST, "build the neighbour lists first");
  if (!eval_supported(s->mdev[slot])) return fail(s, NEP_ERR_UNSUPPORTED, "no compiled kernel for this model shape");
  // the force weights in sorted order go to the sort scratch (free between list builds)
  double* w = nullptr;
  if (gF) {
    HIPCHK(launch_gather_vec64(s->N, s->perm, gF, s->x_alt, s->st));
    w = s->x_alt;
  }
  HIPCHK(launch_grad64(s->mdev[slot], s->m64[slot], eval_buffers(s, slot), w, gE, grad, s->model[slot].n_params,
                       s->st));
  return NEP_OK;
}

int nep_adam_update(nep_system* s, float* theta, const float* grad, float* m1, float* m2, int64_t n, int64_t t,
                    double lr, double beta1, double beta2, double eps) {
  if (!s || !theta || !grad || !m1 || !m2 || n < 1 || t < 1) return fail(s, NEP_ERR_ARG, "bad argument");
  HIPCHK(launch_adam(theta, grad, m1, m2, n, t, lr, beta1, beta2, eps, s->st));
  return NEP_OK;
}

int nep_profile(nep_system* s, int32_t enable) {
  if (!s) return NEP_ERR_ARG;
  if (enable) {
    if (s->pool.empty()) {
      s->pool.resize(kPoolEvents);
      for (auto& e : s->pool) HIPCHK(hipEventCreate(&e));
    }
    int st = prof_drain(s);
    if (st) return st;
    for (int k = 0; k < 6; ++k) {
      s->prof_ms[k] = 0;
      s->prof_cnt[k] = 0;
    }
    s->prof = true;
  } else {
    int st = prof_drain(s);
    if (st) return st;
    s->prof = false;
  }
  return NEP_OK;
}

int nep_profile_read(nep_system* s, double* ms6, int64_t* count6) {
  if (!s || !ms6 || !count6) return NEP_ERR_ARG;
  int st = prof_drain(s);
  if (st) return st;
  for (int k = 0; k < 6; ++k) {
    ms6[k] = s->prof_ms[k];
    count6[k] = s->prof_cnt[k];
  }
  return NEP_OK;
}

int nep_pair_counts(nep_system* s, int64_t* counts3) {
  if (!s || !counts3) return NEP_ERR_ARG;
  if (!s->force_valid[0] && !s->force_valid[1]) return fail(s, NEP_ERR_STALE_LIST, "no evaluation yet");
  HIPCHK(launch_sum_i32(s->N, s->nactR, s->partial, P_ERR2, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_ERR2, 1, s->res + 14, s->st));
  HIPCHK(launch_sum_i32(s->N, s->nactA, s->partial, P_ERR2, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_ERR2, 1, s->res + 15, s->st));
  HIPCHK(launch_sum_i32(s->N, s->cnt, s->partial, P_ERR2, s->st));
  HIPCHK(launch_reduce_partials(s->partial, s->nblocks, P_ERR2, 1, s->res + 16, s->st));
  double r[3];
  HIPCHK(hipMemcpyAsync(r, s->res + 14, 3 * sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  for (int k = 0; k < 3; ++k) counts3[k] = (int64_t)r[k];
  return NEP_OK;
}


// ---------------------------------------------------------------- allocation-free evaluation

int nep_compute_energy_forces_virial_noalloc(const nep_model* model, int64_t n_atoms, const double box[3],
                                             int32_t cap_radial, int32_t cap_angular, double skin, const double* x,
                                             const int32_t* types, int32_t precision, double* energy,
                                             double* virial9, double* forces, double* per_atom_energy,
                                             void* hip_stream) {
  if (!model || !box || !x || !types || !energy || !virial9 || n_atoms < 1 || n_atoms >= kMaxAtoms ||
      cap_radial < 1 || cap_angular < 1 || cap_radial > kMaxCap || cap_angular > kMaxCap || precision < 0 ||
      precision > 2 || !(skin >= 0) || !std::isfinite(skin))
    return NEP_ERR_ARG;
  for (int c = 0; c < 3; ++c)
    if (!(box[c] > 0) || !std::isfinite(box[c])) return NEP_ERR_ARG;
  const double cut = model->hp.rc_radial + skin;
  for (int c = 0; c < 3; ++c)
    if (!(box[c] >= 2.0 * cut)) return NEP_ERR_BOX_TOO_SMALL;
  // the workspace this system needs, carved from the scratch instead of a caller buffer
  nep_system s;
  s.N = n_atoms;
  for (int c = 0; c < 3; ++c) s.box[c] = box[c];
  s.capR = cap_radial;
  s.capA = cap_angular;
  s.model[0].hp = model->hp;  // hyperparameters only: the parameters are read from *model
  s.model[0].D = model->D;
  s.model[0].n_params = model->n_params;
  s.has_model[0] = true;
  s.n_types = model->hp.n_types;
  s.max_ncell = max_cells(box, model->hp.rc_radial);
  const int64_t np[2] = {model->n_params, 0};
  const int HD[2] = {model->hp.n_hidden * model->D, 0};
  if (layout(&s, nullptr, n_atoms, cap_radial, cap_angular, s.max_ncell, np, HD) > kNoallocScratchBytes)
    return NEP_ERR_TOO_LARGE;
  if (hipGetDevice(&s.device) != hipSuccess) return NEP_ERR_HIP;
  void* ws = nullptr;
  int st = noalloc_scratch(s.device, &ws);
  if (st) return st;
  layout(&s, (char*)ws, n_atoms, cap_radial, cap_angular, s.max_ncell, np, HD);
  s.st = (hipStream_t)hip_stream;
  if ((st = upload_model(&s, 0, *model))) return st;
  if (!eval_supported(s.mdev[0])) return NEP_ERR_UNSUPPORTED;
  for (int t = 0; t < kMaxTypes; ++t) {  // masses do not enter the energy or forces
    s.mt.mass[t] = 1.0;
    s.mt.inv_mxi[t] = 1.0 / kXi;
  }
  // state (device arrays in the caller's order), lists with skin, evaluation
  const CellGrid g = make_grid(s.box, model->hp.rc_radial);
  HIPCHK2(launch_zero_i32(s.flags, FLAG_COUNT, s.st));
  HIPCHK2(launch_zero_i32(s.nbr, (int64_t)(cap_radial + kListPad) * n_atoms, s.st));
  HIPCHK2(launch_state_in(n_atoms, x, nullptr, types, s.n_types, g, s.x, s.v, s.type, s.perm, s.pos, s.flags, s.st));
  int32_t f[FLAG_COUNT];
  if ((st = read_flags(&s, f))) return st;
  if (f[FLAG_TYPE]) return NEP_ERR_TYPE;
  if (f[FLAG_NONFINITE]) return NEP_ERR_NONFINITE;
  s.have_state = true;
  if ((st = nep_build_neighbors(&s, skin))) return st;
  return nep_compute_energy_forces_virial(&s, 0, precision, energy, virial9, forces, per_atom_energy, 1);
}

}  // extern "C"
