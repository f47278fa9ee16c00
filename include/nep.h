/*
 * nep.h: C-ABI of the MI355X (gfx950) NEP molecular-dynamics library.
 *
 * The problem (Section III.B and Section VI.A of the paper): given species and
 * positions of atoms in a periodic box, evaluate the neuroevolution potential
 *   U = sum_i U_i,  U_i = sum_mu w1_mu tanh(sum_nu W0_mu,nu q~_nu^i - b0_mu) - b1,
 * its forces and virial, and advance molecular dynamics with neighbour lists
 * that are rebuilt periodically. q^i are radial descriptors (Chebyshev radial
 * functions summed over neighbours inside the radial cutoff) and angular
 * descriptors (radial functions times spherical harmonics, contracted over m,
 * inside the shorter angular cutoff), plus the l = 2 four-body invariant.
 *
 * Conventions for every call:
 *   - Every call returns an int status (enum nep_status) and never aborts or
 *     throws across the ABI. nep_last_error() gives a message for the last
 *     failing call on that system.
 *   - Units: angstrom, femtosecond, eV, amu, kelvin.
 *   - Atom arrays at the boundary are in the caller's ORIGINAL atom order,
 *     row-major [N][3] for vectors. Internally atoms are kept sorted by cell.
 *   - Ownership: the caller owns every host array and the device workspace
 *     (allocated by the caller, e.g. as a torch tensor). The library never
 *     allocates device memory; it only carves the workspace. Pointers are
 *     borrowed for the duration of the call. The system object itself is a
 *     small host allocation freed by nep_system_destroy.
 *   - Ordering: all device work of a system runs in order on the HIP stream
 *     given at creation. Calls that return host values synchronise that
 *     stream before returning; calls whose outputs are device pointers
 *     (on_device = 1) do not synchronise.
 *   - A system handle is not thread-safe.
 *   - Box: orthorhombic and periodic; every side must be at least
 *     2 * (radial cutoff + skin), otherwise NEP_ERR_BOX_TOO_SMALL.
 */
#ifndef NEP_MI355X_H
#define NEP_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nep_model nep_model;
typedef struct nep_system nep_system;

enum nep_status {
  NEP_OK = 0,
  NEP_ERR_ARG = -1,                /* null pointer, bad size or bad value          */
  NEP_ERR_BOX_TOO_SMALL = -2,      /* a side shorter than 2 (cutoff + skin)        */
  NEP_ERR_NEIGHBOR_OVERFLOW = -3,  /* a list exceeded its capacity (results void)  */
  NEP_ERR_TYPE = -4,               /* an atom type outside [0, n_types)            */
  NEP_ERR_NONFINITE = -5,          /* NaN or Inf in positions, forces or energy    */
  NEP_ERR_HIP = -6,                /* a HIP runtime call failed                    */
  NEP_ERR_WORKSPACE = -7,          /* workspace missing, too small or misaligned   */
  NEP_ERR_STALE_LIST = -8,         /* evaluation requested before any list build   */
  NEP_ERR_UNSUPPORTED = -9,        /* model shape without a compiled kernel        */
  NEP_ERR_TOO_LARGE = -10          /* system beyond the allocation-free call's scratch */
};

enum nep_precision {
  NEP_FP32 = 0,  /* descriptors, forces FP32; network FP32 MFMA, FP32 accumulate   */
  NEP_BF16 = 1,  /* as FP32, but the network's matrix operands are bfloat16        */
  NEP_FP64 = 2   /* every operation FP64 from FP64 parameters, for checks (finite
                    differences, reference comparisons): much slower; accepted by
                    nep_compute_energy_forces_virial only                        */
};

/* Model hyperparameters (Section VI.A: n_max 4, basis size 8, three-body
 * l_max 4, four-body l_max 2, 30 hidden neurons; two cutoffs, Fig. 1).
 * n_max_* counts channels 0..n_max, basis_* counts functions 0..basis.
 * l_max_4b is 0 (no four-body term) or 2.
 * Compiled shapes: (n_max 4, basis 8) with either (l_max_3b 4, l_max_4b 2,
 * n_hidden 30) or (l_max_3b 2, l_max_4b 0, n_hidden 8); n_types 1 or 2. */
typedef struct nep_hparams {
  int32_t n_types;
  int32_t n_max_radial, n_max_angular;
  int32_t basis_radial, basis_angular;
  int32_t l_max_3b, l_max_4b;
  int32_t n_hidden;
  double rc_radial, rc_angular;  /* rc_angular <= rc_radial */
  /* ZBL screened-Coulomb repulsion (Section VI.A adds it to the Cu and HfO2
   * models with an outer cutoff): zbl_rc_outer = 0 leaves it out; otherwise
   * 0 <= zbl_rc_inner < zbl_rc_outer <= rc_radial, and each pair closer than
   * zbl_rc_outer adds the universal ZBL energy of atomic numbers zbl_z[t_i],
   * zbl_z[t_j] (> 0), switched off by a cosine between the two radii, half to
   * each atom's energy. It has no trainable parameters. */
  double zbl_rc_inner, zbl_rc_outer;
  double zbl_z[2];
} nep_hparams;

/* Packed FP64 parameter vector, in this order:
 *   cR    [T][T][n_max_R+1][basis_R+1]  radial coefficients, (center type, neighbour type)
 *   cA    [T][T][n_max_A+1][basis_A+1]  angular coefficients
 *   sigma [D]                           descriptor scaler, q~ = q * sigma
 *   W0    [H][D]                        hidden weights, row = hidden unit
 *   b0    [H], w1 [H], b1 [1]
 * with D = (n_max_R+1) + (n_max_A+1) l_max_3b + (l_max_4b == 2 ? n_max_A+1 : 0) and
 * descriptor order [radial n | angular l = 1..l_max_3b, each n | four-body n]. */
int nep_param_count(const nep_hparams* hp, int64_t* n_params, int32_t* n_desc);

/* Create a host-side model (validated copy of hp and params). */
int nep_model_create(const nep_hparams* hp, const double* params, int64_t n_params,
                     nep_model** out);
void nep_model_destroy(nep_model* m);

/* Bytes of device workspace a system needs. surrogate may be NULL; otherwise it
 * has the full model's number of species and cutoffs no larger than the full
 * model's (it reads the full model's lists, visiting only their distance bins up to
 * its own cutoffs), else NEP_ERR_ARG; nep_system_create checks the same.
 * n_atoms: 1 .. 2^28 - 1 (list entries carry a 4-bit distance bin above the
 * 28-bit atom index while the lists are built); cap_radial, cap_angular: 1 .. 4096.
 * cap_radial / cap_angular: per-atom capacities of the lists with skin
 * (radial cutoff + skin, angular cutoff + skin). */
int nep_system_workspace_bytes(const nep_model* full, const nep_model* surrogate,
                               int64_t n_atoms, const double box[3], int32_t cap_radial,
                               int32_t cap_angular, int64_t* bytes);

/* Create a system on the current HIP device. workspace: device pointer,
 * 256-byte aligned, at least nep_system_workspace_bytes long, owned by the
 * caller and kept alive until nep_system_destroy. hip_stream: a hipStream_t
 * (NULL = default stream). The models' parameters are copied into the
 * workspace; the models may be destroyed afterwards. */
int nep_system_create(const nep_model* full, const nep_model* surrogate, int64_t n_atoms,
                      const double box[3], int32_t cap_radial, int32_t cap_angular,
                      void* workspace, int64_t workspace_bytes, void* hip_stream,
                      nep_system** out);
void nep_system_destroy(nep_system* s);

/* Replace one model's parameters (slot 0 = full, 1 = surrogate) from host FP64,
 * same hyperparameters as at creation. */
int nep_system_set_params(nep_system* s, int32_t slot, const double* params, int64_t n_params);

/* Set positions x [N][3] (inside [0, L) per axis), velocities v [N][3] (NULL = zero),
 * types [N] and masses per type [n_types] (amu, host). on_device = 1: x, v,
 * types are device pointers. Invalidates the neighbour lists. */
int nep_set_state(nep_system* s, const double* x, const double* v, const int32_t* types,
                  const double* masses, int32_t on_device);

/* Sort atoms by cell and build the lists with skin (Section VI.A neighbour
 * buffer; 27-cell stencil): radial r^2 < (rc_radial+skin)^2, angular
 * r^2 < (rc_angular+skin)^2, FP64 minimum-image distances. Synchronises.
 * Returns NEP_ERR_NEIGHBOR_OVERFLOW (message gives the needed capacities). */
int nep_build_neighbors(nep_system* s, double skin);

/* Copy a list out (which 0 = radial, 1 = angular) as CSR over ORIGINAL ids,
 * each row ascending: offsets [N+1] and idx [cap_total] (host). */
int nep_export_neighbors(nep_system* s, int32_t which, int64_t* offsets, int32_t* idx,
                         int64_t cap_total);

/* Energy, virial and (optionally) forces and per-atom energies at the current
 * positions (Section III.B: the total energy is the sum of the per-atom network
 * outputs U_i of the descriptors q^i, and the forces F_i = sum_j (dU_i/dr_ij -
 * dU_j/dr_ji) and the virial follow from the derivatives of U_i with respect to
 * the pair vectors r_ij = x_j - x_i), for model slot 0 (full) or 1 (surrogate), with precision
 * NEP_FP32, NEP_BF16 or NEP_FP64 (checks only). energy, virial9 (row-major 3x3,
 * W_ab = -sum_i sum_j (r_ij)_a (dU_i/dr_ij)_b) are host pointers and always
 * written (FP64 reductions on the device). forces [N][3] and per_atom_energy
 * [N] (FP64, original order) may be NULL; on_device says whether they are
 * device pointers. Requires a built list whose skin still covers the current
 * positions (nep_step keeps it so). Synchronises. */
int nep_compute_energy_forces_virial(nep_system* s, int32_t slot, int32_t precision,
                                     double* energy, double* virial9, double* forces,
                                     double* per_atom_energy, int32_t on_device);

/* Advance n_steps of FP64 velocity Verlet with step dt_fs (Section VI.A uses
 * 1 fs). Lists are rebuilt at every rebuild_every-th step and early whenever
 * any atom moved more than skin/2 since the last build. mts_k = 0: plain
 * velocity Verlet with the full model. mts_k >= 1: multiple time stepping with
 * the surrogate as the fast force and the full model applied every mts_k
 * steps (n_steps must be a multiple of mts_k); when the surrogate's force
 * error against the full model exceeds fallback_rms or fallback_max (eV/A, or
 * multiples of the block's rms full-model force after nep_set_judge(s, 1)),
 * the next blocks fall back to the full model until 10 blocks in a row pass.
 * precision: NEP_FP32 or NEP_BF16. With a thermostat set (nep_set_thermostat)
 * the steps are NVT and mts_k must be 0. The list flags are checked after
 * every rebuild_every-th step and after every MTS block: a list that overflowed
 * its capacity at a build stops the run at the first such check with
 * NEP_ERR_NEIGHBOR_OVERFLOW (at most rebuild_every steps, or one block, after
 * the build); the state is that of the step reached (nep_get_state), the
 * steps since the overflowing build used truncated lists and are void, and
 * the next call rebuilds the lists. thermo (host, nullable):
 * rows of 8 doubles {step, potential, kinetic, temperature, pressure (eV/A^3),
 * surrogate rms error, surrogate max error, fallback flag} every thermo_every
 * steps (and the final step), at most max_rows rows. Synchronises at the end,
 * after each MTS block and when the thermo buffer fills. */
int nep_step(nep_system* s, int64_t n_steps, double dt_fs, int32_t rebuild_every, double skin,
             int32_t mts_k, double fallback_rms, double fallback_max, int32_t precision,
             double* thermo, int32_t thermo_every, int64_t max_rows, int64_t* rows_written);

/* NVT. With chain_length >= 1, nep_step (mts_k = 0) integrates velocity Verlet
 * with a Nose-Hoover chain of that many thermostats (at most 16) at the target
 * temperature (K) with period tau_fs (fs): chain masses Q_1 = Nf kT tau^2 and
 * Q_k = kT tau^2, Nf = 3N - 3, and a chain half step (the explicit reversible
 * Trotter form of Martyna, Tuckerman, Tobias and Klein, 1996) before the first
 * and after the second half kick of every step. The application run of Section
 * VII uses the NVT ensemble without naming its thermostat. chain_length = 0
 * returns to NVE. Every call resets the chain state to zero. nep_step refuses
 * mts_k > 0 while a thermostat is set. Synchronises. */
int nep_set_thermostat(nep_system* s, double temperature, double tau_fs, int32_t chain_length);

/* Restores a chain state (host arrays of chain_length values, as returned by
 * nep_get_thermostat) after nep_set_thermostat, to resume an NVT run from a
 * checkpoint together with nep_set_state. Synchronises. */
int nep_set_thermostat_state(nep_system* s, const double* eta, const double* v_eta);

/* The chain state (host arrays of chain_length values, nullable) and its share
 * of the conserved energy, Nf kT eta_1 + kT sum_{k>=2} eta_k + sum_k Q_k v_k^2 / 2
 * (eV, nullable); PE + KE + that share is conserved by the NVT dynamics.
 * Synchronises. */
int nep_get_thermostat(nep_system* s, double* eta, double* v_eta, double* chain_energy);

/* How nep_step's MTS judge reads fallback_rms and fallback_max: relative = 0
 * (the default) takes them in eV/A; relative = 1 takes them as multiples of
 * the per-component rms of the full model's forces at the end of the block
 * being judged, so the test follows the force scale as the system heats or
 * disorders. It changes only the fallback decision. */
int nep_set_judge(nep_system* s, int32_t relative);

/* Order of the force accumulation for every later evaluation and step
 * (Section III.B: F_i gathers dU_i/dr_ij from its own pair terms and -dU_j/dr_ji
 * from each neighbour j's). deterministic = 0 (the default): each center adds its
 * angular terms to its neighbours with atomic additions, so the order of the FP32
 * sums, and the last bits of the forces, can change from run to run.
 * deterministic = 1: no atomics; every atom sums its own terms and then, in list
 * order, the angular terms of its neighbours, each recomputed from that
 * neighbour's dU/ds; the same list, positions and model then give bitwise the
 * same forces, energy and virial on every run. It costs a second pass over the
 * angular lists in the force kernel. Energies are unchanged; forces agree with
 * the default mode to FP32 rounding. Returns NEP_ERR_ARG for other values.
 * Systems created while the environment variable NEP_DETERMINISTIC is "1" start
 * in deterministic mode. */
int nep_set_deterministic(nep_system* s, int32_t deterministic);

/* Positions and velocities [N][3] in original order, and the step counter. */
int nep_get_state(nep_system* s, double* x, double* v, int64_t* step, int32_t on_device);

/* Counters since creation: {list builds, MTS blocks, fallback blocks, steps}. */
int nep_get_stats(nep_system* s, int64_t* stats4);

/* Force-halo tables of the last list build (host int64 stats4): {workgroup tiles
 * of 256 cell-sorted atoms, tiles whose halo does not fit the force kernel's LDS
 * copy (more than 3,840 atoms, 512 cells, or a tile spanning more than 48 cells)
 * and therefore scatter their angular reaction forces with global atomics (the
 * consolidated three-body backward of Section V.B, Optimization 1, without the
 * LDS stage), the largest halo in atoms and in cells over the tiles whose tables
 * were built}. Requires a built list (NEP_ERR_STALE_LIST). Synchronises. */
int nep_halo_stats(nep_system* s, int64_t* stats4);

/* ---------------------------------------------------------------- training
 * Differentiation of E and F with respect to the network parameters
 * theta = (W0 [H][D], b0 [H], w1 [H], b1), packed FP32 in that order on the
 * device (H*D + 2H + 1 values). These calls use the descriptor coefficients
 * and scaler of the model in the given slot and the current positions and
 * lists; the network parameters come from theta.
 *
 * nep_train_forward: E (host FP64) and forces F [N][3] (device FP32, original
 * order) for theta.
 * nep_train_backward: grad = dL/dtheta (device FP32, FP64 reduction over atoms)
 * for L = gE * E + sum_i gF_i . F_i, with gF [N][3] device FP32 in original order
 * (NULL = no force term); accumulate = 1 adds to grad instead of overwriting it.
 * It must follow nep_train_forward (or an evaluation) of the same slot at the
 * same positions, whose pair lists it reuses. Does not synchronise. */
int nep_train_forward(nep_system* s, int32_t slot, const float* theta, double* energy,
                      float* forces);
int nep_train_backward(nep_system* s, int32_t slot, const float* theta, double gE,
                       const float* gF, float* grad, int32_t accumulate);

/* The same with respect to every parameter of the model (Section III.B names
 * the expansion coefficients c of the radial functions trainable): params and
 * grad are device FP32 vectors of n_params values in the packed order of
 * nep_model_create, [cR | cA | sigma | W0 | b0 | w1 | b1]. The forward call
 * evaluates the model with all parameters taken from params; the backward call
 * writes (or, with accumulate = 1, adds) dL/dparams, including dL/dc and the
 * gradient with respect to the descriptor scaler sigma (a caller that keeps
 * sigma fixed ignores that block). The gradient kernels use the system's
 * partial-sum buffer, so calls on one system must not overlap. The same
 * ordering rules as nep_train_backward apply. Does not synchronise. */
int nep_train_forward_params(nep_system* s, int32_t slot, const float* params, double* energy,
                             float* forces);
int nep_train_backward_params(nep_system* s, int32_t slot, const float* params, double gE,
                              const float* gF, float* grad, int32_t accumulate);

/* FP64 form of nep_train_backward_params, for checks: grad = dL/dparams for
 * L = gE * E + sum_i gF_i . F_i, with E and F those of the NEP_FP64 evaluation of
 * the slot's own parameters (as given to nep_model_create or
 * nep_system_set_params) at the current positions and lists, so that central
 * differences of that evaluation's L check it (Section III.B: the expansion
 * coefficients c are trainable; the descriptor scaler sigma and the network
 * weights likewise). Every descriptor, JVP, network and gradient term is FP64;
 * one thread per center, sums over atoms with FP64 atomics (the last bits
 * depend on their order). gF: [N][3] device FP64 in original order, or NULL
 * for no force term. grad: device FP64, n_params values in the packed order
 * [cR | cA | sigma | W0 | b0 | w1 | b1], overwritten. Uses the sort scratch and
 * the system's stream; does not synchronise. Returns NEP_ERR_STALE_LIST
 * without a list and NEP_ERR_UNSUPPORTED for model shapes without a compiled
 * kernel (those of the FP32 path). */
int nep_train_backward64(nep_system* s, int32_t slot, double gE, const double* gF, double* grad);

/* One Adam step on device FP32 arrays theta, grad, m1, m2 of length n
 * (t = 1-based step count), on the system's stream. */
int nep_adam_update(nep_system* s, float* theta, const float* grad, float* m1, float* m2,
                    int64_t n, int64_t t, double lr, double beta1, double beta2, double eps);

/* Force error of the surrogate against the full model at the current positions:
 * err2 = {rms, max} over atoms of |F_full - F_surrogate| (host). */
int nep_surrogate_error(nep_system* s, int32_t precision, double* err2);

/* ---------------------------------------------------------------- measurement
 * nep_profile(s, 1) starts timing kernels with HIP events recorded on the
 * system's stream; nep_profile(s, 0) stops. nep_profile_read returns, since
 * enabling, the summed milliseconds and the number of timed launches of six
 * groups: {descriptor + network kernel of slot 0, force kernel of slot 0, list
 * rebuild (conditional kernels included), integrator kernels, descriptor +
 * network kernel of slot 1, force kernel of slot 1}. Reading synchronises. */
int nep_profile(nep_system* s, int32_t enable);
int nep_profile_read(nep_system* s, double* ms6, int64_t* count6);

/* Pair counts summed over atoms at the last evaluation: counts3 = {radial pairs
 * (r < rc_radial), angular pairs (r < rc_angular), radial list entries with skin}. */
int nep_pair_counts(nep_system* s, int64_t* counts3);

/* ---------------------------------------------------------------- allocation-free call
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): energy, virial and forces of one
 * configuration, as nep_system_create + nep_set_state + nep_build_neighbors +
 * nep_compute_energy_forces_virial would give them (same kernels), but with the system's
 * workspace carved from a fixed device scratch of 64 MiB that the library holds on every
 * GPU it runs on until the process ends, instead of a caller-owned buffer. The call
 * allocates no device memory (no hipMalloc, no allocating library routine); the caller
 * still owns the inputs and outputs.
 *   model: as for nep_system_create (no surrogate). n_atoms, box, cap_radial, cap_angular,
 *   skin: as for nep_system_create and nep_build_neighbors. x [N][3] (FP64) and types [N]
 *   (int32) are DEVICE arrays in the caller's atom order. precision: NEP_FP32, NEP_BF16 or
 *   NEP_FP64. energy and virial9 are host pointers; forces [N][3] and per_atom_energy [N]
 *   (FP64, caller's order) are device pointers and may be NULL. hip_stream: a hipStream_t
 *   (NULL = default stream); the call synchronises it.
 * Errors: NEP_ERR_TOO_LARGE when the system's workspace (about 2.8 KB per atom at
 * capacities 160/96, so roughly 23,000 atoms) exceeds the scratch, checked before any
 * device work; the other codes as for the calls it replaces. Every call on a GPU uses that
 * GPU's one scratch and leaves its contents behind (each call clears what it needs), so
 * calls that overlap on one GPU (different streams or host threads) race: serialise them. */
int nep_compute_energy_forces_virial_noalloc(const nep_model* model, int64_t n_atoms, const double box[3],
                                             int32_t cap_radial, int32_t cap_angular, double skin,
                                             const double* x, const int32_t* types, int32_t precision,
                                             double* energy, double* virial9, double* forces,
                                             double* per_atom_energy, void* hip_stream);

const char* nep_status_string(int status);
const char* nep_last_error(const nep_system* s);

#ifdef __cplusplus
}
#endif

#endif /* NEP_MI355X_H */
