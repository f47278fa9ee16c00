// Internal declarations shared by the HIP translation units of libnep.
// Not part of the public ABI (see include/nep.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace nep {

constexpr int kBlock = 256;          // threads per workgroup for per-atom kernels
constexpr int kMaxTypes = 2;
constexpr int kNumXcd = 8;           // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kPartialStride = 16;   // doubles per workgroup in reduction partials

// Energy/virial partial slots.
enum { P_ENERGY = 0, P_VIR = 1 /* 9 values */, P_KE = 10, P_ERR2 = 11, P_ERRMAX = 12, P_MAXD2 = 13, P_F2 = 14 };

// Device flag words (int32).
enum {
  FLAG_OVF_R = 0,      // max radial list length seen (atomicMax)
  FLAG_OVF_A = 1,      // max angular list length seen
  FLAG_TYPE = 2,       // type out of range
  FLAG_NONFINITE = 3,  // NaN/Inf seen
  FLAG_REBUILD = 4,    // 1 = the current step rebuilds its lists
  FLAG_NBUILD = 5,     // number of list builds (device counter)
  FLAG_BIN_A = 6,      // last distance bin of the angular pairs an evaluation of model 0 visits
  FLAG_BIN_R = 7,      // last distance bin of the radial pairs an evaluation of model 0 visits
  FLAG_BIN_A1 = 8,     // the same for model 1 (the surrogate, whose cutoffs may be shorter)
  FLAG_BIN_R1 = 9,
  FLAG_COUNT = 10
};

// Each atom has one neighbour list with skin (r < rc_radial + skin), ordered by the
// distance at build time into bins. The bin edges are the angular edges
// rc_angular + f_k skin and the radial edges rc_radial + f_k skin (f_k = bin_frac(k)),
// merged, sorted and without duplicates; bin b holds the pairs with
// E[b-1] <= r < E[b]. The angular candidates are therefore a prefix of the list.
// Between rebuilds a distance changes by at most twice the largest displacement d
// since the build, so an evaluation visits the radial pairs up to the edge
// rc_radial + f_k skin and the angular pairs up to rc_angular + f_k skin for the
// first k with f_k skin >= 2 d; every visited pair is still tested against the
// true cutoff. The edges come from both models' cutoffs (at most kMaxBins; beyond
// that the largest skin fractions are dropped, the surrogate's first), and each
// model visits the bins up to the first edges at or beyond its own.
// bp[b][i] = number of entries of atom i in bins 0..b.
constexpr int kFracs = 5;
__host__ __device__ constexpr float bin_frac(int k) {
  return k == 0 ? 0.f : (k == 1 ? 0.05f : (k == 2 ? 0.15f : (k == 3 ? 0.35f : 1.0f)));
}
constexpr int kMaxBins = 16;  // distinct edges of both models' cutoffs; bins fit in 4 bits
struct BinEdges {
  double e2[kMaxBins];       // squared edges, ascending; e2[nbins - 1] = (rc_radial + skin)^2, then infinity
  int nbins;
  int idxR[2][kFracs];       // per model: first bin whose upper edge is >= rc_radial + f_k skin
  int idxA[2][kFracs];       // per model: the same for rc_angular + f_k skin
};

// Orthorhombic cell grid over the box. Cells are numbered brick by brick: bricks
// of 2 x 2 x 2 cells in row-major brick order, cells inside a brick in row-major
// order, so that consecutive cell ids (and the cell-sorted atoms of a 256-atom
// tile) stay spatially compact. ncell counts brick slots (8 per brick); slots past
// an odd grid edge hold no atoms.
struct CellGrid {
  int nc[3];
  int nb[3];
  int ncell;
  double box[3];
};

__host__ __device__ inline int cell_lin(const CellGrid& g, int cx, int cy, int cz) {
  const int b = ((cz >> 1) * g.nb[1] + (cy >> 1)) * g.nb[0] + (cx >> 1);
  return (b << 3) | ((cz & 1) << 2) | ((cy & 1) << 1) | (cx & 1);
}

// Cell coordinates of a cell id; false for brick slots outside the grid.
__host__ __device__ inline bool cell_coords(const CellGrid& g, int lin, int& cx, int& cy, int& cz) {
  const int b = lin >> 3;
  cx = 2 * (b % g.nb[0]) + (lin & 1);
  cy = 2 * ((b / g.nb[0]) % g.nb[1]) + ((lin >> 1) & 1);
  cz = 2 * (b / (g.nb[0] * g.nb[1])) + ((lin >> 2) & 1);
  return cx < g.nc[0] && cy < g.nc[1] && cz < g.nc[2];
}

// Force halo of a 256-atom tile (one workgroup of the force kernel): the non-empty
// cells within one cell of a cell holding tile atoms, sorted by cell id, so their
// atom ranges increase. Built once per list build; the angular list carries each
// neighbour's index inside its tile's halo.
// Rows of the slot-major neighbour list beyond its capacity. The evaluation loops load the
// indices of the next entries before they know whether those exist, so the list carries
// kListPad extra rows, and every row of it always holds an index of an atom of the system
// (the list is zero-filled when the system is created; a build overwrites entries with
// other atoms' indices), so that such loads and the record loads that follow stay in bounds.
constexpr int kListPad = 4;
constexpr int kTileCellsMax = 48;     // cells a tile may touch
constexpr int kCandMax = 2048;        // >= 27 * kTileCellsMax, power of two
constexpr int kHaloCellsMax = 512;    // cells per halo
// atoms per halo held in LDS: 3840 keeps the force kernel's LDS (halo forces and
// tables, 52 KB) within a third of a CU's 160 KB, so three workgroups fit where the
// registers allow it; FCC boxes at metallic density need at most ~3,400
constexpr int kHaloMax = 3840;
constexpr uint16_t kNoLocal = 0xffff; // tile without an LDS halo
struct HaloTables {
  int32_t* info;   // [ntiles][4] = {ncells, natoms, ok, 0}
  int32_t* start;  // [ntiles][kHaloCellsMax] first sorted atom of each halo cell
  int32_t* off;    // [ntiles][kHaloCellsMax + 1] local offset of each halo cell
};

// Neighbour positions and records, laid out so that every writer stores whole cache
// lines and every gather touches as few 16-byte words as possible:
// pos [N] (16 bytes per atom) = (qx, qy, qz, 0): the position as three 32-bit fractions
//   of the box, q = round(x 2^32 / L) modulo 2^32, so that the two's-complement
//   difference of two atoms' fractions is their minimum-image separation in units of
//   L / 2^32 (the quantum: 1.7e-7 A in a 723 A box). Written by the integrator (and the
//   state upload and list build), gathered by the descriptor pass.
// rec [N][4] (64 bytes per atom), written whole by the descriptor kernel for its own atom
//   and gathered by the force pass: word 0 = (qx, qy, qz, v), the position again and one
//   radial force coefficient; words 1, 2 = eight more radial force coefficients; word 3
//   is zero.
// The FP64 positions stay in the [3][N] position array (integration, list build, ZBL).
// The coefficients are written by the descriptor kernel: for one species
// v = w_0 + sum_k w_k and w_1..w_8 (w_k = sum_n (dU/dq_n) c_nk), with several species
// dU/dq_0..dU/dq_4 in v, w_1..w_4.
__host__ __device__ inline double box_quantum(double L) { return L * (1.0 / 4294967296.0); }
__device__ __forceinline__ uint32_t box_fraction(double x, double L) {
  const double f = rint(x * (4294967296.0 / L));  // in [0, 2^32] for x in [0, L)
  return (uint32_t)(uint64_t)f;                   // 2^32, the image of 0, wraps to 0
}
// Atom i's entry of the position array.
__device__ __forceinline__ void pos_put(uint4* pos, int64_t i, double x, double y, double z, const double* box) {
  pos[i] = make_uint4(box_fraction(x, box[0]), box_fraction(y, box[1]), box_fraction(z, box[2]), 0u);
}

// Outputs of the list build.
struct ListOut {
  int32_t* nbr;     // [capR][N] neighbour list with skin, ordered by distance bin
  int32_t* cnt;     // [N]
  int32_t* bp;      // [kMaxBins][N] cumulative bin breakpoints
  uint16_t* nbrl;   // [capR][N] halo-local index of each entry
  uint16_t* selfl;  // [N] halo-local index of the atom itself
};

// Per-build scratch: each atom's candidates in stencil order, sixteen per segment
// ([ceil(capR / 16)][N][16]): entries as q | bin << 28 (64-byte segments) and their
// 16-bit halo-local indices (32-byte segments).
struct ListScratch {
  uint4* q;
  uint4* l;
};
constexpr int kPlaceParts = 4;   // lanes per atom in the placement; part h starts at entry 32 h
constexpr int kPartLen = 32;
constexpr int64_t kMaxAtoms = (int64_t)1 << 28;  // list entries keep the bin in bits 28-31
constexpr int kMaxCap = 4096;                     // per-atom list capacity (16-bit bin counters)


// Device copy of one model (FP32 parameters, same packed order as the host FP64
// vector) plus a bfloat16 copy of W0.
struct ModelDev {
  int T, nR, kR, nA, kA, L3, L4, H, D;
  float rcR, rcA;
  double rcR64, rcA64;
  const float* cR;
  const float* cA;
  const float* sigma;
  const float* W0;    // [H][D]
  const float* b0;
  const float* w1;
  const float* b1;
  const uint16_t* W0bf;  // [H][D] bfloat16 bits, rounded from the FP64 parameters
  // Radial coefficient tables derived from cR and cA (one [n][2 basis - 1] block per
  // species pair, see nep_fast.h), built on the device by launch_derive_coeffs from the
  // FP32 coefficients in use; hscratch holds the tables of a parameter vector passed to
  // the training calls.
  const float* hR;
  const float* hA;
  float* hscratch;
  // ZBL repulsion: pairs with r^2 < zbl_o2 (0: no ZBL term), switched between
  // zbl_ri and zbl_ro; per species pair (t_i * T + t_j) k_e Z_i Z_j and 1 / a_ij
  double zbl_o2;
  double zbl_ri, zbl_ro;
  double zbl_kzz[kMaxTypes * kMaxTypes];
  double zbl_ainv[kMaxTypes * kMaxTypes];
};

// Makes the LDS writes of a wavefront's lanes visible to its other lanes: an LDS fence and
// a wavefront barrier (for LDS data private to one wavefront; no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// XCD-aware mapping of a workgroup id to a contiguous tile index: workgroups
// are dispatched round-robin over the 8 dies, so consecutive tiles (which share
// neighbour atoms) are given to the same die and its L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int x = b % kNumXcd;
  const int k = b / kNumXcd;
  const int per = nb / kNumXcd;
  const int rem = nb % kNumXcd;
  return x * per + (x < rem ? x : rem) + k;
}

// Minimum image of one FP64 component, as d = x_j - x_i; if (d > L/2) d -= L;
// else if (d < -L/2) d += L (written as selects, so no branch separates the
// loads of a pair's three components).
__device__ __forceinline__ double min_image(double d, double L) {
  const double half = 0.5 * L;
  const double lo = d + L, hi = d - L;
  return d > half ? hi : (d < -half ? lo : d);
}

inline int grid_blocks(int64_t n, int block = kBlock) {
  return (int)((n + block - 1) / block);
}

// ---------------------------------------------------------------- launchers
// Neighbour lists (nep_neighbors.hip)
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st);
hipError_t launch_rebuild(int64_t N, const CellGrid& g, const BinEdges& be, int capR, int capA,
                          double* x, double* v, int32_t* type, int32_t* perm, double* x_alt,
                          double* v_alt, int32_t* type_alt, int32_t* perm_alt, double* x_build,
                          int32_t* cellid, int32_t* cell_sorted, int32_t* src, int32_t* key,
                          int32_t* cell_count, int32_t* cell_start, int32_t* cell_fill,
                          int32_t* scan_tmp, uint4* pos, const ListOut& lists, HaloTables ht,
                          ListScratch sc, int32_t* flags, hipStream_t st);
// Rows of original ids [o_lo, o_hi), ascending, into rows[(o - o_lo) * cap + k].
hipError_t launch_export(int64_t N, const int32_t* perm, const int32_t* nbr, const int32_t* cnt,
                         int cap, int64_t o_lo, int64_t o_hi, int32_t* rows, int32_t* row_cnt,
                         hipStream_t st);

// Evaluation (nep_eval.hip)
struct EvalBuffers {
  int64_t N;
  double box[3];
  const double* x;       // [3][N]
  const int32_t* type;   // [N]
  const int32_t* nbr;    // [capR][N] neighbour list with skin, in distance bins
  const int32_t* bp;     // [kMaxBins][N] bin breakpoints
  int32_t* nactR;        // [N] pairs inside rc_radial at this evaluation
  int32_t* nactA;        // [N] pairs inside rc_angular
  const uint16_t* nbrl;   // [capR][N] halo-local index of each entry
  const uint16_t* selfl;  // [N] halo-local index of the atom itself
  const int32_t* hinfo;   // halo tables of the last list build (see HaloTables)
  const int32_t* hstart;
  const int32_t* hoff;
  float* U;              // [N]
  uint4* pos;            // [N] box-fraction positions (read)
  uint4* rec;            // [N][4] neighbour records (written by the descriptor kernel)
  float* G;              // [nA * ncomp][N] dU/ds for the angular accumulators
  float* F;              // [3][N] forces (FP32 accumulation)
  double* partial;       // [nblocks][kPartialStride]
  int32_t* flags;
  int flag_r, flag_a;    // flag words holding this model's last radial / angular bin
  int deterministic;     // 1: forces gathered in a fixed order, no atomics (k_force<..., true>)
};
bool eval_supported(const ModelDev& m);
// Floats of the derived radial tables of one model (radial then angular blocks).
int64_t derived_coeff_floats(int T, int nR, int kR, int nA, int kA);
// Derived tables of the coefficients cR, cA (FP32, model layout) into hR, hA.
hipError_t launch_derive_coeffs(int T, int nR, int kR, int nA, int kA, const float* cR, const float* cA, float* hR,
                                float* hA, hipStream_t st);
// ev (nullable): three events recorded before the descriptor kernel, between the
// two kernels and after the force kernel.
hipError_t launch_eval(const ModelDev& m, int precision, const EvalBuffers& b, hipStream_t st,
                       hipEvent_t* ev = nullptr);
int eval_partial_blocks(int64_t N);

// MD and reductions (nep_md.hip)
struct MassTable {
  double mass[kMaxTypes];     // amu
  double inv_mxi[kMaxTypes];  // 1 / (m * xi), xi = 103.642697 eV fs^2 / (amu A^2)
};
hipError_t launch_reduce_partials(const double* partial, int nblocks, int first, int nvals,
                                  double* out, hipStream_t st);
hipError_t launch_max_partials(const double* partial, int nblocks, int slot, double* out,
                               hipStream_t st);
hipError_t launch_kick_drift(int64_t N, double dt, CellGrid g, const float* F, const int32_t* type,
                             MassTable mt, double* x, double* v, uint4* pos, const double* x_build,
                             double half_skin2, int32_t* flags, double* partial, hipStream_t st);
// FLAG_BIN_R / FLAG_BIN_A from the per-workgroup displacement maxima the drift
// kernel left in partial.
// workgroups of k_kick_drift, whose per-workgroup maxima launch_select_bin reads
int kick_drift_blocks(int64_t N);
hipError_t launch_select_bin(const double* partial, int nblocks, int32_t* flags, double skin,
                             const BinEdges& be, hipStream_t st);
hipError_t launch_kick(int64_t N, double dt, const float* F, const int32_t* type, MassTable mt,
                       double* v, hipStream_t st);
hipError_t launch_kick_diff(int64_t N, double dt, const float* Fa, const float* Fb,
                            const int32_t* type, MassTable mt, double* v, hipStream_t st);
// FP64 parameters of one model (the packed FP64 vector on the device), for the
// FP64 evaluation (nep_eval64.hip).
struct Model64 {
  const double* cR;
  const double* cA;
  const double* sigma;
  const double* W0;
  const double* b0;
  const double* w1;
  double b1;
};
// Energy partials, forces F64 [3][N] (sorted order) and virial partials in FP64;
// U64 [N] and Fp64 [D][N] are its per-atom energies and dU/dq.
hipError_t launch_eval64(const ModelDev& m, const Model64& p, const EvalBuffers& b, double* U64, double* Fp64,
                         double* F64, hipStream_t st);
hipError_t launch_scalar_out64(int64_t N, const int32_t* perm, const double* u, double* out, hipStream_t st);
// FP64 gradient of gE E + sum gF . F with respect to the packed parameters (n_params
// values, overwritten), gF_sorted [3][N] in sorted order or null.
hipError_t launch_grad64(const ModelDev& m, const Model64& p, const EvalBuffers& b, const double* gF_sorted,
                         double gE, double* grad, int64_t n_params, hipStream_t st);
hipError_t launch_gather_vec64(int64_t N, const int32_t* perm, const double* aos_orig, double* soa_sorted,
                               hipStream_t st);

// Nose-Hoover chain: at most kMaxChain thermostats; the device state holds
// {eta[kMaxChain], v_eta[kMaxChain], velocity scale}.
constexpr int kMaxChain = 16;
constexpr int kNhcDoubles = 2 * kMaxChain + 1;
// One chain half step of length h from the kinetic energy *ke, then v *= the scale.
hipError_t launch_nhc_half(int64_t N, const double* ke, double* nhc, int M, double kT, double tau, double h,
                           double* v, hipStream_t st);
hipError_t launch_kinetic(int64_t N, const double* v, const int32_t* type, MassTable mt,
                          double* partial, hipStream_t st);
hipError_t launch_force_error(int64_t N, const float* Fa, const float* Fb, double* partial,
                              hipStream_t st);
hipError_t launch_set_flag(int32_t* flags, int idx, int value, hipStream_t st);
hipError_t launch_sum_i32(int64_t N, const int32_t* a, double* partial, int slot, hipStream_t st);
hipError_t launch_state_in(int64_t N, const double* x_aos, const double* v_aos,
                           const int32_t* type_in, int n_types, CellGrid g, double* x, double* v,
                           int32_t* type, int32_t* perm, uint4* pos, int32_t* flags, hipStream_t st);
hipError_t launch_state_out(int64_t N, const int32_t* perm, const double* soa, double* aos,
                            hipStream_t st);
hipError_t launch_forces_out(int64_t N, const int32_t* perm, const float* F, double* aos,
                             hipStream_t st);
hipError_t launch_scalar_out(int64_t N, const int32_t* perm, const float* U, double* out,
                             hipStream_t st);
hipError_t launch_gather_vec_f32(int64_t N, const int32_t* perm, const float* aos_orig,
                                 float* soa_sorted, hipStream_t st);
hipError_t launch_scatter_vec_f32(int64_t N, const int32_t* perm, const float* soa_sorted,
                                  float* aos_orig, hipStream_t st);

// Training (nep_train.hip)
struct TrainBuffers {
  EvalBuffers e;
  const float* theta;    // network parameters, packed W0, b0, w1, b1
  const float* gF;       // [3][N] sorted order, may be null
  double gE;
  float* vjp;            // [D][N] scratch
  float* qs;             // [D][N] scratch
  double* gpart;         // [nblocks][train_grad_stride()] FP64 partial gradients
  float* grad;           // [G] output
  int accumulate;        // 1: grad += result
};
hipError_t launch_train_forward(const ModelDev& m, const float* theta, const EvalBuffers& b,
                                hipStream_t st);
hipError_t launch_train_backward(const ModelDev& m, const TrainBuffers& t, hipStream_t st);
// The same with every parameter taken from a packed FP32 vector
// [cR | cA | sigma | W0 | b0 | w1 | b1] (t.theta) and the gradient written in that order.
hipError_t launch_train_forward_params(const ModelDev& m, const float* params, const EvalBuffers& b,
                                       hipStream_t st);
hipError_t launch_train_backward_params(const ModelDev& m, const TrainBuffers& t, hipStream_t st);
int train_partial_blocks(int64_t N);
int train_grad_stride();
hipError_t launch_adam(float* theta, const float* g, float* m1, float* m2, int64_t n, int64_t t,
                       double lr, double b1, double b2, double eps, hipStream_t st);

}  // namespace nep
