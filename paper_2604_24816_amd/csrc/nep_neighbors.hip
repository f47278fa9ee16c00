// Cell binning, stable sort of atoms by cell, and neighbour-list construction.
//
// Atoms are kept sorted by (cell, original id) so that the atoms one wavefront
// handles, and their neighbours, are contiguous in HBM. Lists are stored
// slot-major ([slot][N]) so that lane i of a wavefront reads the list entry of
// atom i: consecutive lanes touch consecutive words.
//
// Pair membership is decided by r^2 < (cutoff + skin)^2 with FP64 minimum-image
// differences and r^2 = (dx*dx + dy*dy) + dz*dz, evaluated without fused
// multiply-add so that the set is reproducible bit for bit (Section VI.A
// neighbour-list buffer; Fig. 1 radial and angular cutoffs).
#include "nep_common.h"

namespace nep {
namespace {

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}
__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Workgroups of the rebuild kernels. Every rebuild kernel is enqueued each step and
// returns at once when no rebuild is due, so the per-atom and per-cell ones stride over a
// capped grid (a multiple of the 8 dies, so that a workgroup stays on its die): a step
// without a rebuild then dispatches a few thousand workgroups, not one per cell or per
// 256 atoms.
constexpr int kRebuildGrid = 8192;
inline int rebuild_grid(int64_t nblocks) { return (int)(nblocks < kRebuildGrid ? nblocks : kRebuildGrid); }

__device__ __forceinline__ int cell_coord(double xv, double L, int n) {
  int c = (int)(xv * ((double)n / L));
  if (c < 0) c = 0;
  if (c > n - 1) c = n - 1;
  return c;
}

__global__ void k_bin(int64_t N, CellGrid g, const double* __restrict__ x, int32_t* __restrict__ cellid,
                      int32_t* __restrict__ count, const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int cx = cell_coord(x[p], g.box[0], g.nc[0]);
    const int cy = cell_coord(x[N + p], g.box[1], g.nc[1]);
    const int cz = cell_coord(x[2 * N + p], g.box[2], g.nc[2]);
    const int c = cell_lin(g, cx, cy, cz);
    cellid[p] = c;
    atomicAdd(&count[c], 1);
  }
}

// Exclusive scan, phase 1: each 256-thread block scans 1024 elements.
constexpr int kScanPer = 4;
constexpr int kScanTile = kBlock * kScanPer;

__global__ void k_scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out, int n,
                             int32_t* __restrict__ tile_sums, const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  __shared__ int32_t s[kBlock];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  int32_t sum = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    sum += v[k];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    int32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = s[threadIdx.x] - sum;  // exclusive prefix of this thread
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1) tile_sums[blockIdx.x] = s[kBlock - 1];
}

// Phase 2: one block scans the tile sums (any count) in chunks, exclusive.
__global__ void k_scan_sums(int32_t* __restrict__ sums, int nt, int32_t* __restrict__ total,
                            const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  __shared__ int32_t s[kBlock];
  int32_t carry = 0;
  for (int base = 0; base < nt; base += kBlock) {
    const int i = base + threadIdx.x;
    const int32_t v = (i < nt) ? sums[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      int32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nt) sums[i] = carry + s[threadIdx.x] - v;
    const int32_t chunk = s[kBlock - 1];
    __syncthreads();
    carry += chunk;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int n, const int32_t* __restrict__ sums,
                           const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / kScanTile];
}

__global__ void k_scatter(int64_t N, const int32_t* __restrict__ cellid, const int32_t* __restrict__ start,
                          int32_t* __restrict__ fill, const int32_t* __restrict__ perm,
                          int32_t* __restrict__ src, int32_t* __restrict__ key,
                          const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int c = cellid[p];
    const int pos = start[c] + atomicAdd(&fill[c], 1);
    src[pos] = (int32_t)p;
    key[pos] = perm[p];
  }
}

// Within each cell, order atoms by original id. One wavefront per cell: each lane holds
// atoms of the cell, counts the cell's smaller keys (the keys are distinct original ids)
// and moves its atom to that rank, so the result is the stable order whatever order the
// scatter's atomics left. Cells of more than kSortMax atoms (none at metallic densities)
// are sorted by one lane by insertion.
constexpr int kSortMax = 256;
constexpr int kSortWaves = kBlock / 64;

__global__ void __launch_bounds__(kBlock) k_cell_sort(int ncell, const int32_t* __restrict__ start,
                                                      int32_t* __restrict__ key, int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  __shared__ int32_t kk[kSortWaves][kSortMax];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int U = kSortMax / 64;
  for (int c = blockIdx.x * kSortWaves + w; c < ncell; c += gridDim.x * kSortWaves) {  // wave-uniform
    const int a = start[c], n = start[c + 1] - a;
    if (n <= 1) continue;
    if (n > kSortMax) {
      if (lane == 0) {
        for (int i = a + 1; i < a + n; ++i) {
          const int32_t k = key[i], s0 = src[i];
          int j = i - 1;
          while (j >= a && key[j] > k) {
            key[j + 1] = key[j];
            src[j + 1] = src[j];
            --j;
          }
          key[j + 1] = k;
          src[j + 1] = s0;
        }
      }
      continue;
    }
    int32_t mk[U], ms[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = lane + 64 * u;
      mk[u] = l < n ? key[a + l] : 0;
      ms[u] = l < n ? src[a + l] : 0;
      if (l < n) kk[w][l] = mk[u];
    }
    wave_lds_sync();
    int rank[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rank[u] = 0;
    for (int m = 0; m < n; ++m) {
      const int32_t km = kk[w][m];
#pragma unroll
      for (int u = 0; u < U; ++u) rank[u] += km < mk[u] ? 1 : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (lane + 64 * u < n) {
        key[a + rank[u]] = mk[u];
        src[a + rank[u]] = ms[u];
      }
    }
    wave_lds_sync();
  }
}

__global__ void k_permute(int64_t N, const int32_t* __restrict__ src, const int32_t* __restrict__ cellid,
                          const double* __restrict__ x, const double* __restrict__ v,
                          const int32_t* __restrict__ type, const int32_t* __restrict__ perm,
                          double* __restrict__ x2, double* __restrict__ v2, int32_t* __restrict__ type2,
                          int32_t* __restrict__ perm2, double* __restrict__ xb,
                          int32_t* __restrict__ cell_sorted, const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = src[p];
    for (int c = 0; c < 3; ++c) {
      const double xv = x[c * N + s];
      x2[c * N + p] = xv;
      xb[c * N + p] = xv;
      v2[c * N + p] = v[c * N + s];
    }
    type2[p] = type[s];
    perm2[p] = perm[s];
    cell_sorted[p] = cellid[s];
  }
}

// Copy the permuted arrays back to the primary buffers.
__global__ void k_copy_back(int64_t N, const double* __restrict__ x2, const double* __restrict__ v2,
                            const int32_t* __restrict__ type2, const int32_t* __restrict__ perm2,
                            double* __restrict__ x, double* __restrict__ v, int32_t* __restrict__ type,
                            int32_t* __restrict__ perm, uint4* __restrict__ pos, CellGrid g,
                            const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    double xn[3];
    for (int c = 0; c < 3; ++c) {
      xn[c] = x2[c * N + p];
      x[c * N + p] = xn[c];
      v[c * N + p] = v2[c * N + p];
    }
    pos_put(pos, p, xn[0], xn[1], xn[2], g.box);
    type[p] = type2[p];
    perm[p] = perm2[p];
  }
}

// Exclusive prefix sum over the workgroup; returns this thread's prefix, total in *tot.
__device__ __forceinline__ int block_scan(int v, int* scan, int* tot) {
  __syncthreads();
  scan[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int t = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
    __syncthreads();
    scan[threadIdx.x] += t;
    __syncthreads();
  }
  const int incl = scan[threadIdx.x];
  *tot = scan[kBlock - 1];
  return incl - v;
}

// One workgroup per 256-atom tile: the tile's force halo (every non-empty cell within
// one cell, periodic, of a cell holding tile atoms), sorted by cell id, with local
// offsets. ok = 0 when the tile or its halo exceeds the LDS tables of the force kernel.
__device__ void halo_tile(int64_t N, const CellGrid& g, const int32_t* __restrict__ cell_sorted,
                          const int32_t* __restrict__ cell_start, const HaloTables& ht, int tile) {
  __shared__ int cand[kCandMax];
  __shared__ int scan[kBlock];
  __shared__ int cnt[kHaloCellsMax];
  const int64_t t0 = (int64_t)tile * kBlock;
  const int64_t t1 = t0 + kBlock < N ? t0 + kBlock : N;
  int32_t* info = ht.info + 4 * tile;
  const int c_lo = cell_sorted[t0], c_hi = cell_sorted[t1 - 1];
  const int ncr = c_hi - c_lo + 1;
  if (ncr > kTileCellsMax) {
    if (threadIdx.x == 0) {
      info[0] = 0;
      info[1] = 0;
      info[2] = 0;
      info[3] = 0;
    }
    return;
  }
  int n_sort = 64;
  while (n_sort < 27 * ncr) n_sort <<= 1;
  for (int t = threadIdx.x; t < n_sort; t += kBlock) {
    int v = 0x7fffffff;
    if (t < 27 * ncr) {
      const int c = c_lo + t / 27, o = t % 27;
      int cx, cy, cz;
      if (cell_start[c + 1] > cell_start[c] && cell_coords(g, c, cx, cy, cz)) {
        const int nx = (cx + o % 3 - 1 + g.nc[0]) % g.nc[0];
        const int ny = (cy + (o / 3) % 3 - 1 + g.nc[1]) % g.nc[1];
        const int nz = (cz + o / 9 - 1 + g.nc[2]) % g.nc[2];
        v = cell_lin(g, nx, ny, nz);
      }
    }
    cand[t] = v;
  }
  __syncthreads();
  for (int k = 2; k <= n_sort; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < n_sort; t += kBlock) {
        const int u = t ^ j;
        if (u > t) {
          const int a = cand[t], c = cand[u];
          if ((a > c) == ((t & k) == 0)) {
            cand[t] = c;
            cand[u] = a;
          }
        }
      }
      __syncthreads();
    }
  const int per = (n_sort + kBlock - 1) / kBlock;
  const int e0 = threadIdx.x * per;
  int mine = 0;
  for (int e = e0; e < e0 + per && e < n_sort; ++e) {
    const int c = cand[e];
    if (c != 0x7fffffff && (e == 0 || cand[e - 1] != c) && cell_start[c + 1] > cell_start[c]) ++mine;
  }
  int ncells = 0;
  int pos = block_scan(mine, scan, &ncells);
  if (ncells > kHaloCellsMax) {
    if (threadIdx.x == 0) {
      info[0] = 0;
      info[1] = 0;
      info[2] = 0;
      info[3] = 0;
    }
    return;
  }
  int32_t* hs = ht.start + (int64_t)tile * kHaloCellsMax;
  int32_t* ho = ht.off + (int64_t)tile * (kHaloCellsMax + 1);
  for (int e = e0; e < e0 + per && e < n_sort; ++e) {
    const int c = cand[e];
    if (c != 0x7fffffff && (e == 0 || cand[e - 1] != c) && cell_start[c + 1] > cell_start[c]) {
      hs[pos] = cell_start[c];
      cnt[pos] = cell_start[c + 1] - cell_start[c];
      ++pos;
    }
  }
  __syncthreads();
  const int per2 = (ncells + kBlock - 1) / kBlock;
  const int k0 = threadIdx.x * per2;
  int sum = 0;
  for (int k = k0; k < k0 + per2 && k < ncells; ++k) sum += cnt[k];
  int natoms = 0;
  int run = block_scan(sum, scan, &natoms);
  for (int k = k0; k < k0 + per2 && k < ncells; ++k) {
    ho[k] = run;
    run += cnt[k];
  }
  if (threadIdx.x == 0) {
    ho[ncells] = natoms;
    info[0] = ncells;
    info[1] = natoms;
    info[2] = natoms <= kHaloMax ? 1 : 0;
    info[3] = 0;
  }
}

__global__ void __launch_bounds__(kBlock)
k_halo_tables(int64_t N, CellGrid g, const int32_t* __restrict__ cell_sorted,
              const int32_t* __restrict__ cell_start, HaloTables ht, const int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  const int ntiles = (int)((N + kBlock - 1) / kBlock);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    halo_tile(N, g, cell_sorted, cell_start, ht, tile);
    __syncthreads();  // the LDS tables are reused by the next tile
  }
}

// Halo-local index of sorted atom q in tile `tile` (q must lie in the halo).
__device__ __forceinline__ int halo_index(const HaloTables& ht, int tile, int ncells, int q) {
  const int32_t* hs = ht.start + (int64_t)tile * kHaloCellsMax;
  const int32_t* ho = ht.off + (int64_t)tile * (kHaloCellsMax + 1);
  int lo = 0, hi = ncells - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hs[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return ho[lo] + (q - hs[lo]);
}

// Distance bin of a pair inside the list cutoff: the number of interior edges <= r^2,
// testing the first NE edges (the outer edge and the unused ones, set to infinity, are
// never reached; NE >= nbins - 1).
template <int NE>
__device__ __forceinline__ int bin_of(double r2, const BinEdges& be) {
  int k = 0;
#pragma unroll
  for (int m = 0; m < NE; ++m) k += r2 >= be.e2[m] ? 1 : 0;
  return k;
}
// Edge tests of the list build: one model's nine interior edges, or the union of two
// models' edges.
constexpr int kEdgesOne = 2 * kFracs - 1;
constexpr int kEdgesTwo = kMaxBins - 1;

// Pair vector x_q - x_p in FP64 followed by the periodic shift of the stencil cell
// (-L, 0 or +L: the value the minimum-image rule subtracts for every pair that can
// lie within the cutoff when the dimension holds at least three cells), or by the
// minimum-image rule itself when some dimension has fewer cells (MINIMG);
// r^2 = (dx*dx + dy*dy) + dz*dz without FMA.
template <bool MINIMG>
__device__ __forceinline__ double cand_r2(const double* __restrict__ x, int64_t N, int64_t q, double xi, double yi,
                                          double zi, double sx, double sy, double sz, const CellGrid& g) {
#pragma clang fp contract(off)
  double dx = x[q] - xi, dy = x[N + q] - yi, dz = x[2 * N + q] - zi;
  if constexpr (MINIMG) {
    dx = g.nc[0] < 3 ? min_image(dx, g.box[0]) : dx + sx;
    dy = g.nc[1] < 3 ? min_image(dy, g.box[1]) : dy + sy;
    dz = g.nc[2] < 3 ? min_image(dz, g.box[2]) : dz + sz;
  } else {
    dx = dx + sx;
    dy = dy + sy;
    dz = dz + sz;
  }
  const double sxx = dx * dx;
  const double syy = dy * dy;
  const double szz = dz * dz;
  const double sxy = sxx + syy;
  return sxy + szz;
}

// Candidates of one stencil cell, four at a time (their positions are loaded
// together before any is tested).
template <bool MINIMG, class Visit>
__device__ __forceinline__ void scan_cell(const double* __restrict__ x, int64_t N, int q0, int q1, int64_t p,
                                          double xi, double yi, double zi, double sx, double sy, double sz,
                                          const CellGrid& g, double cut2, Visit&& visit) {
  for (int q = q0; q < q1; q += 4) {
    double r2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r2[u] = cand_r2<MINIMG>(x, N, q + u < q1 ? q + u : q1 - 1, xi, yi, zi, sx, sy, sz, g);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u < q1 && q + u != p && r2[u] < cut2) visit(q + u, r2[u]);
  }
}

// kMaxBins 16-bit counters packed in 64-bit registers: a counter update is a shift
// and a few selects and adds instead of a select chain over kMaxBins registers.
struct BinCounts {
  static constexpr int kWords = (kMaxBins + 3) / 4;
  uint64_t w[kWords] = {};
  __device__ __forceinline__ void add(int b) {
    const uint64_t inc = (uint64_t)1 << (16 * (b & 3));
#pragma unroll
    for (int k = 0; k < kWords; ++k) w[k] += (b >> 2) == k ? inc : 0;
  }
  __device__ __forceinline__ int get(int b) const {
    uint64_t v = w[0];
#pragma unroll
    for (int k = 1; k < kWords; ++k) v = (b >> 2) == k ? w[k] : v;
    return (int)((v >> (16 * (b & 3))) & 0xffffu);
  }
};

// Per-thread staging of one scratch column in LDS: entries are collected sixteen
// at a time (stride 17 words, no bank conflicts) and written out as one 64-byte
// segment at [k / 16][atom][16] (or 32 bytes of 16-bit values), so the global
// stores are whole segments even though the threads flush at different times.
constexpr int kStage = 16;
constexpr int kStageStride = kStage + 1;

__device__ __forceinline__ void stage_flush32(const uint32_t* st, uint4* col, int64_t N, int64_t p, int k) {
  uint4* dst = col + ((int64_t)(k / kStage) * N + p) * (kStage / 4);
#pragma unroll
  for (int j = 0; j < kStage / 4; ++j)
    dst[j] = make_uint4(st[4 * j], st[4 * j + 1], st[4 * j + 2], st[4 * j + 3]);
}
__device__ __forceinline__ void stage_flush16(const uint32_t* st, uint4* col, int64_t N, int64_t p, int k) {
  uint4* dst = col + ((int64_t)(k / kStage) * N + p) * (kStage / 8);
#pragma unroll
  for (int j = 0; j < kStage / 8; ++j)
    dst[j] = make_uint4((st[8 * j] & 0xffffu) | (st[8 * j + 1] << 16), (st[8 * j + 2] & 0xffffu) | (st[8 * j + 3] << 16),
                        (st[8 * j + 4] & 0xffffu) | (st[8 * j + 5] << 16), (st[8 * j + 6] & 0xffffu) | (st[8 * j + 7] << 16));
}

// One thread per atom, one pass over the 27-cell stencil. Every candidate inside the
// list cutoff is appended, in stencil order, to the atom's scratch column as
// q | bin << 28 together with its halo-local index. Stencil cells whose nearest point
// lies beyond the list cutoff (with a 1e-6 A margin) are skipped. k_place_lists then
// counts the entries per bin and orders them by bin.
// With MARKED, only the atoms that k_build_cells left to it (cnt = -1) are built.
template <bool MINIMG, int NE, bool MARKED>
__device__ void build_list_atom(int64_t N, const CellGrid& g, const double* __restrict__ x,
                                const int32_t* __restrict__ start, const int32_t* __restrict__ cell_sorted,
                                const BinEdges& be, int capR, const ListOut& lo_, const HaloTables& ht,
                                const ListScratch& sc, int32_t* __restrict__ flags, int64_t p) {
  if (p >= N) return;
  if (MARKED && lo_.cnt[p] != -1) return;
  const int tile = (int)(p / kBlock);
  const bool hok = ht.info[4 * tile + 2] != 0;
  const int hcells = ht.info[4 * tile + 0];
  lo_.selfl[p] = hok ? (uint16_t)halo_index(ht, tile, hcells, (int)p) : kNoLocal;
  const double cut2 = be.e2[be.nbins - 1];
  const double xi = x[p], yi = x[N + p], zi = x[2 * N + p];
  int cx, cy, cz;
  cell_coords(g, cell_sorted[p], cx, cy, cz);
  const int cc3[3] = {cx, cy, cz};
  const double pos3[3] = {xi, yi, zi};
  int lo[3], nof[3];
  double dlo[3], dhi[3];  // distance from the atom to the lower / upper face of its cell
  for (int d = 0; d < 3; ++d) {
    lo[d] = g.nc[d] >= 3 ? -1 : 0;
    nof[d] = g.nc[d] >= 3 ? 3 : g.nc[d];
    const double h = g.box[d] / g.nc[d];
    dlo[d] = fmax(pos3[d] - cc3[d] * h - 1e-6, 0.0);
    dhi[d] = fmax((cc3[d] + 1) * h - pos3[d] - 1e-6, 0.0);
  }
  int n = 0;
  __shared__ uint32_t stage_q[kBlock * kStageStride], stage_l[kBlock * kStageStride];
  uint32_t* sq = stage_q + threadIdx.x * kStageStride;
  uint32_t* sl = stage_l + threadIdx.x * kStageStride;
  for (int a = 0; a < nof[2]; ++a) {
    const int rz = cz + lo[2] + a;
    const int zc = (rz + g.nc[2]) % g.nc[2];
    const double sz = rz < 0 ? -g.box[2] : (rz >= g.nc[2] ? g.box[2] : 0.0);
    const double gz = nof[2] < 3 ? 0.0 : (a == 0 ? dlo[2] : (a == 2 ? dhi[2] : 0.0));
    for (int b = 0; b < nof[1]; ++b) {
      const int ry = cy + lo[1] + b;
      const int yc = (ry + g.nc[1]) % g.nc[1];
      const double sy = ry < 0 ? -g.box[1] : (ry >= g.nc[1] ? g.box[1] : 0.0);
      const double gy = nof[1] < 3 ? 0.0 : (b == 0 ? dlo[1] : (b == 2 ? dhi[1] : 0.0));
      for (int e = 0; e < nof[0]; ++e) {
        const int rx = cx + lo[0] + e;
        const int xc = (rx + g.nc[0]) % g.nc[0];
        const double sx = rx < 0 ? -g.box[0] : (rx >= g.nc[0] ? g.box[0] : 0.0);
        const double gx = nof[0] < 3 ? 0.0 : (e == 0 ? dlo[0] : (e == 2 ? dhi[0] : 0.0));
        if (gx * gx + gy * gy + gz * gz >= cut2) continue;
        const int cc = cell_lin(g, xc, yc, zc);
        const int q0 = start[cc], q1 = start[cc + 1];
        if (q1 <= q0) continue;
        // halo-local index of sorted atom q is loc0 + q (cells are contiguous in the halo)
        const int loc0 = hok ? halo_index(ht, tile, hcells, q0) - q0 : 0;
        scan_cell<MINIMG>(x, N, q0, q1, p, xi, yi, zi, sx, sy, sz, g, cut2, [&](int q, double r2) {
          if (n < capR) {
            sq[n % kStage] = (uint32_t)q | ((uint32_t)bin_of<NE>(r2, be) << 28);
            sl[n % kStage] = hok ? (uint32_t)(loc0 + q) : (uint32_t)kNoLocal;
            if (n % kStage == kStage - 1) {
              stage_flush32(sq, sc.q, N, p, n);
              stage_flush16(sl, sc.l, N, p, n);
            }
          }
          ++n;
        });
      }
    }
  }
  if (n < capR && n % kStage != 0) {
    stage_flush32(sq, sc.q, N, p, n);
    stage_flush16(sl, sc.l, N, p, n);
  }
  lo_.cnt[p] = n < capR ? n : capR;
  if (n > capR) atomicMax(&flags[FLAG_OVF_R], n);
}

template <bool MINIMG, int NE, bool MARKED = false>
__global__ void __launch_bounds__(kBlock)
k_build_lists(int64_t N, CellGrid g, const double* __restrict__ x, const int32_t* __restrict__ start,
              const int32_t* __restrict__ cell_sorted, BinEdges be, int capR, int capA, ListOut lo_,
              HaloTables ht, ListScratch sc, int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  const int nblocks = (int)((N + kBlock - 1) / kBlock);
  for (int b = blockIdx.x; b < nblocks; b += gridDim.x)
    build_list_atom<MINIMG, NE, MARKED>(N, g, x, start, cell_sorted, be, capR, lo_, ht, sc, flags,
                                        (int64_t)xcd_tile(b, nblocks) * kBlock + threadIdx.x);
}

// One workgroup per cell (boxes with at least three cells along every dimension):
// the positions of the 27 stencil cells' atoms are staged in LDS once, in stencil
// order and by sorted index inside a cell, and each wavefront takes the cell's atoms
// in turn, its 64 lanes testing two chunks of 64 candidates at a time (their staged
// positions read together, for the latency). The accepted candidates are
// compacted (ballot and prefix count) into a per-wavefront LDS queue in candidate
// order; only those are binned and written, 64 entries per pass, to the atom's
// scratch column. The scratch therefore holds the same entries in the same order as
// the per-atom kernel writes, with the FP64 distance computed the same way. Cells
// whose stencil holds more than kCellCand atoms mark their atoms (cnt = -1) for
// k_build_lists<false, NE, true>.
constexpr int kCellCand = 1024;  // stencil atoms a workgroup stages in LDS
constexpr int kCellQueue = 192;  // accepted candidates queued per wavefront (two chunks past a drain)

template <int NE>
__device__ void build_cell(int64_t N, const CellGrid& g, const double* __restrict__ x,
                           const int32_t* __restrict__ start, const BinEdges& be, int capR, const ListOut& lo_,
                           const HaloTables& ht, const ListScratch& sc, int32_t* __restrict__ flags, int c) {
#pragma clang fp contract(off)
  const int s0 = start[c], s1 = start[c + 1];
  if (s1 <= s0) return;  // empty cell or brick slot outside the grid
  int cx, cy, cz;
  cell_coords(g, c, cx, cy, cz);
  __shared__ double X[kCellCand], Y[kCellCand], Z[kCellCand];
  __shared__ int32_t Q[kCellCand];
  __shared__ uint8_t C[kCellCand];
  __shared__ int cq0[27], cum[28];
  __shared__ double shift[3][27];
  __shared__ uint32_t qk[kBlock / 64][kCellQueue];
  __shared__ double qr[kBlock / 64][kCellQueue];
  __shared__ int loc0s[2][27];  // halo offset of each stencil cell for the cell's first two tiles
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int tile0 = s0 / kBlock;
  int cnt_s = 0;
  if (t < 27) {  // stencil cell t = 9 a + 3 b + e: z offset a - 1, y offset b - 1, x offset e - 1
    const int r3[3] = {cx + t % 3 - 1, cy + (t / 3) % 3 - 1, cz + t / 9 - 1};
    int w3[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      w3[d] = (r3[d] + g.nc[d]) % g.nc[d];
      shift[d][t] = r3[d] < 0 ? -g.box[d] : (r3[d] >= g.nc[d] ? g.box[d] : 0.0);
    }
    const int cc = cell_lin(g, w3[0], w3[1], w3[2]);
    cq0[t] = start[cc];
    cnt_s = start[cc + 1] - start[cc];
    cum[t] = cnt_s;
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int k = 0; k < 27; ++k) {
      const int v = cum[k];
      cum[k] = acc;
      acc += v;
    }
    cum[27] = acc;
  }
  __syncthreads();
  const int nc = cum[27];
  if (nc > kCellCand) {
    for (int p = s0 + t; p < s1; p += kBlock) lo_.cnt[p] = -1;
    return;
  }
  // halo-local offsets for the tile of the cell's first atom and the next tile if it
  // holds atoms of the cell (other tiles, for cells of more than 256 atoms, are
  // looked up when reached); computed while the positions load
  if (t >= 64 && t < 64 + 54) {
    const int u = t - 64, tl = tile0 + u / 27, sc = u % 27;
    int v = 0;
    if (tl * kBlock < s1 && ht.info[4 * tl + 2] != 0 && cum[sc + 1] > cum[sc])
      v = halo_index(ht, tl, ht.info[4 * tl + 0], cq0[sc]) - cq0[sc];
    loc0s[u / 27][sc] = v;
  }
  for (int k = t; k < nc; k += kBlock) {
    int sidx = 0;
#pragma unroll
    for (int m = 1; m < 27; ++m) sidx += k >= cum[m] ? 1 : 0;
    const int q = cq0[sidx] + (k - cum[sidx]);
    X[k] = x[q];
    Y[k] = x[N + q];
    Z[k] = x[2 * N + q];
    Q[k] = q;
    C[k] = (uint8_t)sidx;
  }
  __syncthreads();
  // a cell away from the periodic boundary has no image shifts
  const bool shifted = cx == 0 || cy == 0 || cz == 0 || cx == g.nc[0] - 1 || cy == g.nc[1] - 1 ||
                       cz == g.nc[2] - 1;
  const double cut2 = be.e2[be.nbins - 1];
  uint32_t* scq = reinterpret_cast<uint32_t*>(sc.q);
  uint16_t* scl = reinterpret_cast<uint16_t*>(sc.l);
  int cached_tile = -1, hok = 0, hcells = 0, loc0 = 0;  // loc0: of stencil cell `lane`, for the atom's tile
  for (int p = s0 + w; p < s1; p += kBlock / 64) {  // wave-uniform
    const int tile = p / kBlock;
    if (tile != cached_tile) {
      cached_tile = tile;
      hcells = ht.info[4 * tile + 0];
      hok = ht.info[4 * tile + 2] != 0;
      loc0 = 0;
      if (tile - tile0 < 2) {
        if (lane < 27) loc0 = loc0s[tile - tile0][lane];
      } else if (hok && lane < 27 && cum[lane + 1] > cum[lane]) {
        loc0 = halo_index(ht, tile, hcells, cq0[lane]) - cq0[lane];
      }
    }
    // the atom lies in its own cell, stencil cell 13
    const int self_off = __shfl(loc0, 13);
    if (lane == 0) lo_.selfl[p] = hok ? (uint16_t)(self_off + p) : kNoLocal;
    const int ks = cum[13] + (p - s0);  // the atom's own slot (stencil cell 13 is its cell)
    const double xi = X[ks], yi = Y[ks], zi = Z[ks];
    int nw = 0, nq = 0;  // entries written, entries queued (wave-uniform)
    auto drain = [&]() {
      wave_lds_sync();
      for (int j0 = 0; j0 < nq; j0 += 64) {
        const int j = j0 + lane;
        const bool v = j < nq;
        const int k = v ? (int)qk[w][j] : 0;
        const int sidx = C[k];
        const int lc = __shfl(loc0, sidx);
        const int e = nw + j;
        if (v && e < capR) {
          const int q = Q[k];
          const int64_t o = ((int64_t)(e / kStage) * N + p) * kStage + e % kStage;
          scq[o] = (uint32_t)q | ((uint32_t)bin_of<NE>(qr[w][j], be) << 28);
          scl[o] = hok ? (uint16_t)(lc + q) : kNoLocal;
        }
      }
      nw += nq;
      nq = 0;
      wave_lds_sync();
    };
    // the FP64 squared distance to stencil slot k, the expression of the per-atom build
    auto dist2 = [&](int k) {
      double dx = X[k] - xi, dy = Y[k] - yi, dz = Z[k] - zi;
      if (shifted) {
        const int sidx = C[k];
        dx = dx + shift[0][sidx];
        dy = dy + shift[1][sidx];
        dz = dz + shift[2][sidx];
      }
      const double sxx = dx * dx;
      const double syy = dy * dy;
      const double szz = dz * dz;
      const double sxy = sxx + syy;
      return sxy + szz;
    };
    // appends the accepted candidates of one 64-candidate chunk, in candidate order
    auto enqueue = [&](int k, bool acc, double r2) {
      const uint64_t m = __ballot(acc);
      const int pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
      if (acc) {
        qk[w][nq + pre] = (uint32_t)k;
        qr[w][nq + pre] = r2;
      }
      nq += __popcll(m);
    };
    // two chunks per pass, their staged positions read together
    for (int k0 = 0; k0 < nc; k0 += 128) {
      const int ka = k0 + lane, kb = k0 + 64 + lane;
      bool acc_a = false, acc_b = false;
      double ra = 0.0, rb = 0.0;
      if (ka < nc && ka != ks) {
        ra = dist2(ka);
        acc_a = ra < cut2;
      }
      if (kb < nc && kb != ks) {
        rb = dist2(kb);
        acc_b = rb < cut2;
      }
      enqueue(ka, acc_a, ra);
      enqueue(kb, acc_b, rb);
      if (nq > kCellQueue - 128) drain();
    }
    drain();
    if (lane == 0) {
      lo_.cnt[p] = nw < capR ? nw : capR;
      if (nw > capR) atomicMax(&flags[FLAG_OVF_R], nw);
    }
  }
}

template <int NE>
__global__ void __launch_bounds__(kBlock)
k_build_cells(int64_t N, CellGrid g, const double* __restrict__ x, const int32_t* __restrict__ start,
              BinEdges be, int capR, ListOut lo_, HaloTables ht, ListScratch sc, int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  for (int cb = blockIdx.x; cb < g.ncell; cb += gridDim.x) {
    build_cell<NE>(N, g, x, start, be, capR, lo_, ht, sc, flags, xcd_tile(cb, g.ncell));
    __syncthreads();  // the LDS staging is reused by the next cell
  }
}

// One wavefront per 16 atoms, four lanes per atom: counts each atom's scratch
// entries per bin, writes the bin breakpoints, and orders the entries by bin (stable
// inside a bin), writing the list and its halo-local indices row by row, 16
// consecutive atoms (64 bytes) per store, through LDS tiles of kPlaceRows rows;
// longer lists take further rounds. Lane h counts and places entries [32 h, 32 (h + 1))
// (the last lane the rest), starting each bin after the entries of earlier parts.
// Entries outside the current round go to a spare row.
constexpr int kPlaceRows = 159;  // one round for lists up to 159 entries (FCC metals at 7 A: ~135-150)
constexpr int kPlaceAtoms = 64 / kPlaceParts;
constexpr int kPlaceGrid = 16384;  // workgroups of the placement (grid-stride over atom groups)

__global__ void __launch_bounds__(64)
k_place_lists(int64_t N, int nbins, int binA, int capR, int capA, ListOut lo_, ListScratch sc,
              int32_t* __restrict__ flags) {
  if (flags[FLAG_REBUILD] == 0) return;
  __shared__ uint32_t tile[(kPlaceRows + 1) * kPlaceAtoms];
  __shared__ uint16_t ltile[(kPlaceRows + 1) * kPlaceAtoms];
  __shared__ uint16_t off[kMaxBins * 64];  // next position of each bin, per lane
  __shared__ uint64_t parts[kPlaceParts][BinCounts::kWords][kPlaceAtoms];  // per-bin counts of each part
  const int lane = threadIdx.x;
  const int a = lane % kPlaceAtoms;  // atom of the wavefront
  const int h = lane / kPlaceAtoms;  // which part of its column
  // groups of kPlaceAtoms atoms, strided over a capped grid: a step without a rebuild
  // then dispatches few workgroups
  const int64_t ngroups = (N + kPlaceAtoms - 1) / kPlaceAtoms;
  // the list length of the lane's atom in the next group is loaded one group ahead
  int cnt_next = (int64_t)blockIdx.x * kPlaceAtoms + a < N ? lo_.cnt[(int64_t)blockIdx.x * kPlaceAtoms + a] : 0;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t p = grp * kPlaceAtoms + a;
    const bool valid = p < N;
    const int cnt = valid ? cnt_next : 0;
    {
      const int64_t pn = (grp + gridDim.x) * kPlaceAtoms + a;
      cnt_next = grp + gridDim.x < ngroups && pn < N ? lo_.cnt[pn] : 0;
    }
    const int g_lo = h * kPartLen;
    const int g_hi = h == kPlaceParts - 1 ? cnt : (g_lo + kPartLen < cnt ? g_lo + kPartLen : cnt);
    const bool work = valid && g_lo < cnt;
    // longest list of the wavefront (uniform loop bounds for the row writes)
    int rows_max = cnt;
  #pragma unroll
    for (int o = 32; o > 0; o >>= 1) rows_max = max(rows_max, __shfl_xor(rows_max, o, 64));
    // per-bin counts of this lane's part (16-bit fields), then of the parts before it
    // and of the whole list
    // this lane's part of the scratch column: the first two 16-entry chunks stay in
    // registers from the counting pass to the placement (parts hold 32 entries, the last
    // part the rest), later chunks are read again
    auto load_q = [&](int g, uint32_t* v) {
      const uint4* src = sc.q + ((int64_t)(g / kStage) * N + p) * (kStage / 4);
  #pragma unroll
      for (int j = 0; j < kStage / 4; ++j) {
        const uint4 w = src[j];
        v[4 * j] = w.x;
        v[4 * j + 1] = w.y;
        v[4 * j + 2] = w.z;
        v[4 * j + 3] = w.w;
      }
    };
    // the halo indices of a chunk, 16-bit, as two 16-byte words
    auto load_l = [&](int g, uint4* lw) {
      const uint4* ls = sc.l + ((int64_t)(g / kStage) * N + p) * (kStage / 8);
  #pragma unroll
      for (int j = 0; j < kStage / 8; ++j) lw[j] = ls[j];
    };
    BinCounts mine;
    auto count_chunk = [&](int g, const uint32_t* v) {
  #pragma unroll
      for (int u = 0; u < kStage; ++u)
        if (g + u < g_hi) mine.add((int)(v[u] >> 28));
    };
    uint32_t c0[kStage], c1[kStage];
    uint4 l0[kStage / 8], l1[kStage / 8];  // their halo indices, loaded with them
    const bool two = work && g_lo + kStage < g_hi;
    if (work) {
      load_q(g_lo, c0);
      load_l(g_lo, l0);
      if (two) {
        load_q(g_lo + kStage, c1);
        load_l(g_lo + kStage, l1);
      }
      count_chunk(g_lo, c0);
      if (two) count_chunk(g_lo + kStage, c1);
      for (int g = g_lo + 2 * kStage; g < g_hi; g += kStage) {
        uint32_t t[kStage];
        load_q(g, t);
        count_chunk(g, t);
      }
    }
  #pragma unroll
    for (int k = 0; k < BinCounts::kWords; ++k) parts[h][k][a] = mine.w[k];
    __syncthreads();
    BinCounts before, total;
  #pragma unroll
    for (int q = 0; q < kPlaceParts; ++q)
  #pragma unroll
      for (int k = 0; k < BinCounts::kWords; ++k) {
        const uint64_t c = parts[q][k][a];
        total.w[k] += c;
        before.w[k] += q < h ? c : 0;
      }
    // bin breakpoints (cumulative counts); angular candidates are the bins up to binA
    int bstart[kMaxBins];
    {
      int t = 0;
  #pragma unroll
      for (int k = 0; k < kMaxBins; ++k) {
        bstart[k] = t;
        t += k < nbins ? total.get(k) : 0;
        if (valid && h == 0 && k < nbins) lo_.bp[(int64_t)k * N + p] = t < capR ? t : capR;
        if (valid && h == 0 && k == binA && t > capA) atomicMax(&flags[FLAG_OVF_A], t);
      }
    }
    constexpr int rows = kPlaceRows;  // row `rows` of the tiles is the spare row
    for (int r0 = 0; r0 < rows_max; r0 += rows) {
      if (work) {
  #pragma unroll
        for (int k = 0; k < kMaxBins; ++k) off[k * 64 + lane] = (uint16_t)(bstart[k] + before.get(k));
        auto place_chunk = [&](int g, const uint32_t* v, const uint4* lw) {
          uint32_t hl[kStage];
  #pragma unroll
          for (int j = 0; j < kStage / 8; ++j) {
            const uint4 w = lw[j];
            const uint32_t t[4] = {w.x, w.y, w.z, w.w};
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              hl[8 * j + 2 * u] = t[u] & 0xffffu;
              hl[8 * j + 2 * u + 1] = t[u] >> 16;
            }
          }
  #pragma unroll
          for (int u = 0; u < kStage; ++u) {
            const bool live = g + u < g_hi;
            const int oi = (int)(v[u] >> 28) * 64 + lane;
            int pos = -1;
            if (live) {
              pos = off[oi];
              off[oi] = (uint16_t)(pos + 1);
            }
            pos -= r0;
            const int slot = (live && pos >= 0 && pos < rows ? pos : rows) * kPlaceAtoms + a;
            tile[slot] = v[u] & 0x0fffffffu;
            ltile[slot] = (uint16_t)hl[u];
          }
        };
        place_chunk(g_lo, c0, l0);
        if (two) place_chunk(g_lo + kStage, c1, l1);
        for (int g = g_lo + 2 * kStage; g < g_hi; g += kStage) {
          uint32_t t[kStage];
          uint4 lt[kStage / 8];
          load_q(g, t);
          load_l(g, lt);
          place_chunk(g, t, lt);
        }
      }
      __syncthreads();
      // the kPlaceParts lane groups write interleaved rows
      const int nrow = rows_max - r0 < rows ? rows_max - r0 : rows;
      for (int r = h; r < nrow; r += kPlaceParts) {
        if (valid && r0 + r < cnt) {
          lo_.nbr[(int64_t)(r0 + r) * N + p] = (int32_t)tile[r * kPlaceAtoms + a];
          lo_.nbrl[(int64_t)(r0 + r) * N + p] = ltile[r * kPlaceAtoms + a];
        }
      }
      __syncthreads();
    }
    __syncthreads();  // the LDS tiles are reused by the next group
  }
}

// After a build the positions equal the build positions: displacement 0, bin 0.
__global__ void k_count_build(int32_t* flags, int bin_r0, int bin_a0, int bin_r1, int bin_a1) {
  if (flags[FLAG_REBUILD] != 0 && threadIdx.x == 0) {
    flags[FLAG_NBUILD] += 1;
    flags[FLAG_BIN_R] = bin_r0;
    flags[FLAG_BIN_A] = bin_a0;
    flags[FLAG_BIN_R1] = bin_r1;
    flags[FLAG_BIN_A1] = bin_a1;
  }
}

// Lists in original ids, one row per original atom in [o_lo, o_hi), ascending.
__global__ void k_export(int64_t N, const int32_t* __restrict__ perm, const int32_t* __restrict__ nbr,
                         const int32_t* __restrict__ cnt, int cap, int64_t o_lo, int64_t o_hi,
                         int32_t* __restrict__ rows, int32_t* __restrict__ row_cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int64_t o = perm[p];
  if (o < o_lo || o >= o_hi) return;
  const int n = cnt[p] < cap ? cnt[p] : cap;
  int32_t* row = rows + (o - o_lo) * cap;
  for (int k = 0; k < n; ++k) {
    const int32_t val = perm[nbr[(int64_t)k * N + p]];
    int j = k - 1;
    while (j >= 0 && row[j] > val) {
      row[j + 1] = row[j];
      --j;
    }
    row[j + 1] = val;
  }
  row_cnt[o - o_lo] = n;
}

}  // namespace

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_blocks(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f32, dim3(grid_blocks(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_blocks(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

// Every kernel below returns at once when flags[FLAG_REBUILD] == 0, so the whole
// rebuild can be enqueued each step and skipped on the device without a host sync.
hipError_t launch_rebuild(int64_t N, const CellGrid& g, const BinEdges& be, int capR, int capA,
                          double* x, double* v, int32_t* type, int32_t* perm, double* x_alt,
                          double* v_alt, int32_t* type_alt, int32_t* perm_alt, double* x_build,
                          int32_t* cellid, int32_t* cell_sorted, int32_t* src, int32_t* key,
                          int32_t* cell_count, int32_t* cell_start, int32_t* cell_fill,
                          int32_t* scan_tmp, uint4* pos, const ListOut& lout, HaloTables ht,
                          ListScratch sc, int32_t* flags, hipStream_t st) {
  const int nb = grid_blocks(N);
  const int ncell = g.ncell;
  hipError_t e;
  if ((e = launch_zero_i32(cell_count, ncell, st)) != hipSuccess) return e;
  if ((e = launch_zero_i32(cell_fill, ncell, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, g, x, cellid, cell_count, flags);
  const int ntiles = (ncell + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, st, cell_count, cell_start, ncell,
                     scan_tmp, flags);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, st, scan_tmp, ntiles, cell_start + ncell,
                     flags);
  hipLaunchKernelGGL(k_scan_add, dim3(grid_blocks(ncell)), dim3(kBlock), 0, st, cell_start, ncell,
                     scan_tmp, flags);
  hipLaunchKernelGGL(k_scatter, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, cellid, cell_start, cell_fill, perm,
                     src, key, flags);
  hipLaunchKernelGGL(k_cell_sort, dim3(rebuild_grid(grid_blocks(ncell, kSortWaves))), dim3(kBlock), 0, st, ncell,
                     cell_start, key, src, flags);
  hipLaunchKernelGGL(k_permute, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, src, cellid, x, v, type, perm,
                     x_alt, v_alt, type_alt, perm_alt, x_build, cell_sorted, flags);
  hipLaunchKernelGGL(k_copy_back, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, x_alt, v_alt, type_alt, perm_alt,
                     x, v, type, perm, pos, g, flags);
  hipLaunchKernelGGL(k_halo_tables, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, g, cell_sorted, cell_start, ht, flags);
  // the minimum-image rule inside the candidate loop only for boxes with fewer than
  // three cells along some dimension
  const bool small = g.nc[0] < 3 || g.nc[1] < 3 || g.nc[2] < 3;
  const bool one = be.nbins - 1 <= kEdgesOne;
  if (small) {
    auto kern = one ? k_build_lists<true, kEdgesOne> : k_build_lists<true, kEdgesTwo>;
    hipLaunchKernelGGL(kern, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, g, x, cell_start, cell_sorted, be, capR, capA,
                       lout, ht, sc, flags);
  } else {
    auto cells = one ? k_build_cells<kEdgesOne> : k_build_cells<kEdgesTwo>;
    hipLaunchKernelGGL(cells, dim3(rebuild_grid(ncell)), dim3(kBlock), 0, st, N, g, x, cell_start, be, capR, lout, ht, sc,
                       flags);
    // atoms of cells whose stencil did not fit in LDS
    auto rest = one ? k_build_lists<false, kEdgesOne, true> : k_build_lists<false, kEdgesTwo, true>;
    hipLaunchKernelGGL(rest, dim3(rebuild_grid(nb)), dim3(kBlock), 0, st, N, g, x, cell_start, cell_sorted, be, capR, capA,
                       lout, ht, sc, flags);
  }
  const int place_groups = grid_blocks(N, kPlaceAtoms);
  hipLaunchKernelGGL(k_place_lists, dim3(place_groups < kPlaceGrid ? place_groups : kPlaceGrid), dim3(64), 0, st,
                     N, be.nbins,
                     be.idxA[0][kFracs - 1], capR, capA, lout, sc, flags);
  hipLaunchKernelGGL(k_count_build, dim3(1), dim3(64), 0, st, flags, be.idxR[0][0], be.idxA[0][0], be.idxR[1][0],
                     be.idxA[1][0]);
  return hipGetLastError();
}

hipError_t launch_export(int64_t N, const int32_t* perm, const int32_t* nbr, const int32_t* cnt,
                         int cap, int64_t o_lo, int64_t o_hi, int32_t* rows, int32_t* row_cnt,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_export, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, nbr, cnt, cap, o_lo,
                     o_hi, rows, row_cnt);
  return hipGetLastError();
}

}  // namespace nep
