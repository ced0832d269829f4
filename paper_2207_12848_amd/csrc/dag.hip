// Dependency-graph construction for the transport sweep (gfx950).
//
// Compiled with -ffp-contract=off: the face orientation s = (Ox nx + Oy ny) + Oz nz
// must round exactly as written so that every kernel here (and any FP64
// implementation of the same expression) classifies each face identically.
//
//   k_count   per task (unit, cell): upwind/downwind counts, Aperp, boundary outflow
//   k_kahn    per unit, one workgroup: levels by Kahn's algorithm (algorithm 2's
//             counters), ready cells compacted with wavefront ballots
//   k_gather_len, k_fill  row lengths and rows of the upwind/downwind lists,
//             stored in schedule order so a level's rows are contiguous (and
//             Aperp in schedule order, for the per-call preparation)
#include <hipcub/hipcub.hpp>

#include <type_traits>

#include "internal.h"
#include "sweep.h"

namespace sweep {

namespace {

constexpr int kCountBlock = 256;
// k_count: 512 threads (16 directions of a 32-cell tile at a time) so that two
// workgroups with their face tiles and staged rows keep 16 wavefronts per CU
constexpr int kCountThreads = 512;
constexpr int kTileCells = 32;  // cells per tile of the cell-order kernels
// Workgroup of Kahn's algorithm: 15 worker wavefronts and one that stores the
// schedule (the largest workgroup).  A level's frontier is processed in rounds
// of one task per worker thread, each round a chain of dependent memory round
// trips (row loads, then counter decrements), so a typical level of a few
// hundred tasks takes one round.
constexpr int kKahnBlock(int) { return 1024; }

__device__ __forceinline__ double orient(double ox, double oy, double oz, const double* n) {
  const double a = ox * n[0];
  const double b = oy * n[1];
  const double c = oz * n[2];
  return (a + b) + c;
}

// Face weight w = A |Omega . n| from the FP64 orientation s, rounded once to
// FP32: within one rounding of the FP64 weight however grazing the face is (a
// weight formed from FP32 normals would carry an absolute error of ~1e-7 A,
// large against A |s| for nearly parallel faces).  Twin half-faces have equal
// areas and exactly negated normals, so their s differ only in sign and both
// sides of a face get the same weight: what a cell sends through a face is
// exactly what its neighbour receives.
__device__ __forceinline__ float face_w(double A, double s) { return (float)(A * fabs(s)); }

// Unit of block b (units own consecutive block ranges).
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2
// cache: this renumbering gives each XCD one contiguous range of the grid, so
// the workgroups an XCD runs together belong to few units and share those
// units' arrays in its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int kXcd = 8;
  const int per = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd;
  return x * per + min(x, rem) + b / kXcd;
}

__device__ __forceinline__ int unit_of_block(const int32_t* blk_base, int n_units, int b) {
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk_base[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The cell-order kernel stages a tile of kTileCells consecutive cells' faces
// in LDS with coalesced loads (room for kTileFaces faces per cell on average,
// above the ~15.5 of a Voronoi cell and small enough for three workgroups per CU;
// a tile with more faces is read from global memory instead); the workgroup
// then covers every direction, 32 consecutive lanes handling the tile's cells
// for one direction.
constexpr int kTileFaces = 17;

struct FaceTile {
  int c0, cend;       // cells [c0, cend) of mesh m
  int64_t f0;         // first face of the tile
  bool in_lds;        // the tile's faces are in LDS
  const int64_t* fp;  // LDS copy of face_ptr[c0 .. cend] (relative to f0)
};

__host__ __device__ inline size_t tile_lds_bytes() {
  const size_t cap = (size_t)kTileCells * kTileFaces;
  return (8 * (kTileCells + 1) + cap * (24 + 8 + 4 + 1) + 15) / 16 * 16;
}

__device__ __forceinline__ FaceTile stage_tile(const MeshDev& M, int c0, unsigned char* smem) {
  FaceTile T;
  T.c0 = c0;
  T.cend = min(c0 + kTileCells, M.n_cells);
  const int nc = T.cend - c0;
  T.f0 = M.face_ptr[c0];
  const int nf = (int)(M.face_ptr[T.cend] - T.f0);
  constexpr int cap = kTileCells * kTileFaces;
  T.in_lds = nf <= cap;
  int64_t* fp = reinterpret_cast<int64_t*>(smem);
  for (int i = threadIdx.x; i <= nc; i += blockDim.x) fp[i] = M.face_ptr[c0 + i] - T.f0;
  if (T.in_lds) {
    double* nrm = reinterpret_cast<double*>(fp + kTileCells + 1);
    double* area = nrm + 3 * cap;
    int32_t* nbr = reinterpret_cast<int32_t*>(area + cap);
    int8_t* shift = reinterpret_cast<int8_t*>(nbr + cap);
    for (int i = threadIdx.x; i < 3 * nf; i += blockDim.x) nrm[i] = M.face_normal[3 * T.f0 + i];
    for (int i = threadIdx.x; i < nf; i += blockDim.x) {
      area[i] = M.face_area[T.f0 + i];
      nbr[i] = M.face_nbr[T.f0 + i];
      shift[i] = M.face_shift != nullptr ? M.face_shift[T.f0 + i] : (int8_t)0;
    }
  }
  T.fp = fp;
  return T;
}

// Per task: upwind/downwind counts, Aperp = sum of outflow w, boundary outflow
// weights, the signed weight of every face and the fixed-width row of downwind
// cells.  A row holds
// dn_width entries padded with -1; a task with more downwind cells keeps
// dn_width - 1 of them and stores -(o + 2) in the last slot, o being the
// offset in dn_ovf of [count, rest of the list].  A thread handles one cell of
// the tile for one direction; the rows of kCountBlock / kTileCells directions
// are assembled in LDS and written out as contiguous blocks (STAGE), or
// written straight to global memory.
template <bool STAGE>
__global__ __launch_bounds__(kCountThreads) void k_count(DagBuildArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_max[2];
  __shared__ unsigned long long s_ent[2];
  if (threadIdx.x < 2) {
    s_max[threadIdx.x] = 0;
    s_ent[threadIdx.x] = 0ull;
  }
  const int m = a.cblk_mesh[blockIdx.x];
  const MeshDev M = a.meshes[m];
  const FaceTile T = stage_tile(M, a.cblk_c0[blockIdx.x], smem);
  const int W = a.dn_width;
  int32_t* srow = reinterpret_cast<int32_t*>(smem + tile_lds_bytes());
  __syncthreads();
  const int ci = threadIdx.x % kTileCells;
  const int dj = threadIdx.x / kTileCells;
  constexpr int kDirs = kCountThreads / kTileCells;
  const int c = T.c0 + ci;
  const int nc = T.cend - T.c0;
  const bool cell = c < T.cend;
  const int fb = cell ? (int)T.fp[ci] : 0, fe = cell ? (int)T.fp[ci + 1] : 0;
  int mi = 0, mo = 0;
  unsigned long long eu = 0, ed = 0;  // row entries of the thread's tasks
  auto run = [&](const double* nrm, const double* area, const int32_t* nbr, const int8_t* shift) {
    for (int d0 = 0; d0 < a.D; d0 += kDirs) {
      const int d = d0 + dj;
      if (cell && d < a.D) {
        const double ox = a.dirs[3 * d], oy = a.dirs[3 * d + 1], oz = a.dirs[3 * d + 2];
        const int64_t t = a.units[m * a.D + d].task_base + c;
        int32_t* row = STAGE ? srow + threadIdx.x * W : a.dnw + t * W;  // LDS: [dj][ci][W]
        int32_t* ovf = nullptr;
        int nup = 0, ndn = 0;
        double ap = 0.0, wall = 0.0, per = 0.0;
        for (int f = fb; f < fe; ++f) {
          const double* n = nrm + 3 * f;
          const double sv = orient(ox, oy, oz, n);
          const int nb = nbr[f];
          const bool periodic = shift != nullptr && shift[f] != 0;
          const float w = face_w(area[f], sv);
          if (sv > a.eps) {
            ap += w;
            if (nb < 0) wall += w;
            else if (periodic) {
              per += w;
            } else {
              if (ndn < W) {
                row[ndn] = nb;
              } else {
                if (ndn == W) {  // the row is full: continue in an overflow list
                  const int need = (fe - fb) + 2;
                  const int o = atomicAdd(a.dn_ovf_top, need);
                  // a pool that has run out gets the list in its spare end (the
                  // host sees the count past the capacity and redoes the counts)
                  ovf = a.dn_ovf + (o + need <= a.dn_ovf_cap ? o : a.dn_ovf_cap);
                  ovf[1] = row[W - 1];
                  row[W - 1] = -(o + 2);
                }
                ovf[1 + ndn - (W - 1)] = nb;
              }
              ++ndn;
            }
          } else if (sv < -a.eps && nb >= 0 && !periodic) {
            ++nup;
          }
        }
        if (ovf != nullptr) ovf[0] = ndn - (W - 1);
        if (nup >= 15) a.big[atomicAdd(a.big_top, 1)] = t;  // counter too large for 4 bits
        for (int q = ndn; q < W; ++q) row[q] = -1;
        a.indeg[t] = nup;
        a.rowlen_dn[t] = ndn;
        a.aperp[t] = (float)ap;
        a.bnd[t] = make_float2((float)wall, (float)per);
        mi = max(mi, nup);
        mo = max(mo, ndn);
        eu += (unsigned long long)nup;
        ed += (unsigned long long)ndn;
      }
      // the signed weight of every face of the tile for these directions (NaN:
      // neither inflow nor outflow), consecutive threads on consecutive faces
      const int nft = (int)T.fp[nc];
      for (int i = threadIdx.x; i < kDirs * nft; i += kCountThreads) {
        const int j = i / nft, f = i - j * nft;
        const int dd = d0 + j;
        if (dd < a.D) {
          const double sv = orient(a.dirs[3 * dd], a.dirs[3 * dd + 1], a.dirs[3 * dd + 2], nrm + 3 * f);
          const float w = face_w(area[f], sv);
          a.wface[(int64_t)a.D * M.face_off + (int64_t)dd * M.n_faces + T.f0 + f] =
              sv > a.eps ? w : (sv < -a.eps ? -w : __int_as_float(0x7fc00000));
        }
      }
      if (STAGE) {
        __syncthreads();
        // the tile's rows of direction d0 + j are nc * W consecutive ints of dnw
        const int per4 = nc * W / 4;
        for (int i = threadIdx.x; i < kDirs * per4; i += kCountThreads) {
          const int j = i / per4, r = i - j * per4;
          if (d0 + j < a.D) {
            const int64_t tb = a.units[m * a.D + d0 + j].task_base;
            reinterpret_cast<int4*>(a.dnw + (tb + T.c0) * W)[r] =
                reinterpret_cast<const int4*>(srow + j * kTileCells * W)[r];
          }
        }
        __syncthreads();
      }
    }
  };
  if (T.in_lds) {
    constexpr int cap = kTileCells * kTileFaces;
    const double* nrm = reinterpret_cast<const double*>(T.fp + kTileCells + 1);
    const double* area = nrm + 3 * cap;
    const int32_t* nbr = reinterpret_cast<const int32_t*>(area + cap);
    const int8_t* shift = reinterpret_cast<const int8_t*>(nbr + cap);
    run(nrm, area, nbr, shift);
  } else {
    run(M.face_normal + 3 * T.f0, M.face_area + T.f0, M.face_nbr + T.f0,
        M.face_shift != nullptr ? M.face_shift + T.f0 : nullptr);
  }
  atomicMax(&s_max[0], mi);
  atomicMax(&s_max[1], mo);
  atomicAdd(&s_ent[0], eu);
  atomicAdd(&s_ent[1], ed);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(a.stats, s_max[0]);
    atomicMax(a.stats + 1, s_max[1]);
    atomicAdd(a.ent_tot, s_ent[0]);
    atomicAdd(a.ent_tot + 1, s_ent[1]);
  }
}

// Transport scheme (b) (direction-conserving transport, sec. 2.6), per task:
// the cell's outflow Aperp phi is shared equally by its n = min(n_aligned,
// outflow faces) outflow faces with the largest s (ties: the lower face
// index), each carrying w_b = Aperp / n.  Those faces get the signed weight
// +w_b, every other face NaN (nothing leaves through it); they are the task's
// only downwind edges (rows of at most n entries), and the boundary sums count
// only them.  Upwind counts depend on the neighbours' choices and are made by
// k_count_in once every choice is written.
__device__ __forceinline__ void top_insert(double (&bs)[kMaxAligned], int (&bf)[kMaxAligned],
                                           double v, int f) {
  // bs descending; an equal value already present stays first (lower face index)
  const double os[kMaxAligned] = {bs[0], bs[1], bs[2], bs[3]};
  const int of[kMaxAligned] = {bf[0], bf[1], bf[2], bf[3]};
#pragma unroll
  for (int k = 0; k < kMaxAligned; ++k) {
    const bool keep = os[k] >= v;
    const bool from_above = !keep && k > 0 && os[k > 0 ? k - 1 : 0] < v;
    bs[k] = keep ? os[k] : (from_above ? os[k > 0 ? k - 1 : 0] : v);
    bf[k] = keep ? of[k] : (from_above ? of[k > 0 ? k - 1 : 0] : f);
  }
}

__global__ __launch_bounds__(kCountThreads) void k_count_aligned(DagBuildArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_max;
  __shared__ unsigned long long s_ent;
  if (threadIdx.x == 0) {
    s_max = 0;
    s_ent = 0ull;
  }
  const int m = a.cblk_mesh[blockIdx.x];
  const MeshDev M = a.meshes[m];
  const FaceTile T = stage_tile(M, a.cblk_c0[blockIdx.x], smem);
  const int W = a.dn_width;
  __syncthreads();
  const int ci = threadIdx.x % kTileCells;
  const int dj = threadIdx.x / kTileCells;
  constexpr int kDirs = kCountThreads / kTileCells;
  const int c = T.c0 + ci;
  const bool cell = c < T.cend;
  const int fb = cell ? (int)T.fp[ci] : 0, fe = cell ? (int)T.fp[ci + 1] : 0;
  int mo = 0;
  unsigned long long ed = 0;
  auto run = [&](const double* nrm, const double* area, const int32_t* nbr, const int8_t* shift) {
    for (int d0 = 0; d0 < a.D; d0 += kDirs) {
      const int d = d0 + dj;
      if (!(cell && d < a.D)) continue;
      const double ox = a.dirs[3 * d], oy = a.dirs[3 * d + 1], oz = a.dirs[3 * d + 2];
      const int64_t t = a.units[m * a.D + d].task_base + c;
      float* wf = a.wface + (int64_t)a.D * M.face_off + (int64_t)d * M.n_faces + T.f0;
      double ap = 0.0;
      int nout = 0;
      double bs[kMaxAligned];
      int bf[kMaxAligned];
#pragma unroll
      for (int k = 0; k < kMaxAligned; ++k) {
        bs[k] = -__builtin_huge_val();
        bf[k] = -1;
      }
      for (int f = fb; f < fe; ++f) {
        const double sv = orient(ox, oy, oz, nrm + 3 * f);
        if (sv > a.eps) {
          ap += face_w(area[f], sv);
          ++nout;
          top_insert(bs, bf, sv, f);
        }
      }
      const int n = min(nout, a.n_aligned);
      const float wb = n > 0 ? (float)(ap / n) : 0.0f;
      int32_t* row = a.dnw + t * W;
      int ndn = 0;
      double wall = 0.0, per = 0.0;
      for (int f = fb; f < fe; ++f) {
        bool chosen = false;
#pragma unroll
        for (int k = 0; k < kMaxAligned; ++k) chosen |= k < n && bf[k] == f;
        wf[f] = chosen ? wb : __int_as_float(0x7fc00000);
        if (!chosen) continue;
        const int nb = nbr[f];
        if (nb < 0) wall += wb;
        else if (shift != nullptr && shift[f] != 0) {
          per += wb;
        } else {
          row[ndn++] = nb;
        }
      }
      for (int q = ndn; q < W; ++q) row[q] = -1;
      a.aperp[t] = (float)ap;
      a.bnd[t] = make_float2((float)wall, (float)per);
      a.rowlen_dn[t] = ndn;
      mo = max(mo, ndn);
      ed += (unsigned long long)ndn;
    }
  };
  if (T.in_lds) {
    constexpr int cap = kTileCells * kTileFaces;
    const double* nrm = reinterpret_cast<const double*>(T.fp + kTileCells + 1);
    const double* area = nrm + 3 * cap;
    const int32_t* nbr = reinterpret_cast<const int32_t*>(area + cap);
    const int8_t* shift = reinterpret_cast<const int8_t*>(nbr + cap);
    run(nrm, area, nbr, shift);
  } else {
    run(M.face_normal + 3 * T.f0, M.face_area + T.f0, M.face_nbr + T.f0,
        M.face_shift != nullptr ? M.face_shift + T.f0 : nullptr);
  }
  atomicMax(&s_max, mo);
  atomicAdd(&s_ent, ed);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(a.stats + 1, s_max);
    atomicAdd(a.ent_tot + 1, s_ent);
  }
}

// Scheme (b), per task: the upwind dependencies are the faces whose twin the
// neighbour chose (its signed weight is not NaN); counts, row lengths and the
// tasks with 15 or more dependencies, as k_count does for scheme (a).
__global__ __launch_bounds__(kCountThreads) void k_count_in(DagBuildArgs a) {
  __shared__ int s_max;
  __shared__ unsigned long long s_ent;
  if (threadIdx.x == 0) {
    s_max = 0;
    s_ent = 0ull;
  }
  __syncthreads();
  const int m = a.cblk_mesh[blockIdx.x];
  const MeshDev M = a.meshes[m];
  const int ci = threadIdx.x % kTileCells;
  const int dj = threadIdx.x / kTileCells;
  constexpr int kDirs = kCountThreads / kTileCells;
  const int c = a.cblk_c0[blockIdx.x] + ci;
  int mi = 0;
  unsigned long long eu = 0;
  if (c < M.n_cells) {
    const int64_t fb = M.face_ptr[c], fe = M.face_ptr[c + 1];
    for (int d = dj; d < a.D; d += kDirs) {
      const float* wf = a.wface + (int64_t)a.D * M.face_off + (int64_t)d * M.n_faces;
      int nup = 0;
      for (int64_t f = fb; f < fe; ++f) {
        if (M.face_nbr[f] < 0) continue;
        if (isnan(wf[M.face_twin[f]])) continue;
        if (M.face_shift == nullptr || M.face_shift[f] == 0) ++nup;
      }
      const int64_t t = a.units[m * a.D + d].task_base + c;
      if (nup >= 15) a.big[atomicAdd(a.big_top, 1)] = t;  // counter too large for 4 bits
      a.indeg[t] = nup;
      mi = max(mi, nup);
      eu += (unsigned long long)nup;
    }
  }
  atomicMax(&s_max, mi);
  atomicAdd(&s_ent, eu);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(a.stats, s_max);
    atomicAdd(a.ent_tot, s_ent);
  }
}

// Tasks with 15 or more upwind dependencies keep their counter in global
// memory; the entries that point at them in their upwind cells' downwind rows
// get bit 30 set, so that Kahn's algorithm sends those decrements there without
// first reading the LDS counter.  One thread per such task (rare).
constexpr int32_t kBigFlag = 0x40000000;

__global__ void k_mark(DagBuildArgs a, int32_t n_big) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_big) return;
  const int64_t t = a.big[i];
  int lo = 0, hi = a.n_units - 1;  // unit of task t (task bases ascend)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.units[mid].task_base <= t) lo = mid; else hi = mid - 1;
  }
  const Unit U = a.units[lo];
  const int c = (int)(t - U.task_base);
  const MeshDev M = a.meshes[U.mesh];
  const double ox = a.dirs[3 * U.dir], oy = a.dirs[3 * U.dir + 1], oz = a.dirs[3 * U.dir + 2];
  const int W = a.dn_width;
  const float* wf = a.wface + (int64_t)a.D * M.face_off + (int64_t)U.dir * M.n_faces;
  for (int64_t f = M.face_ptr[c]; f < M.face_ptr[c + 1]; ++f) {
    const int nb = M.face_nbr[f];
    if (nb < 0 || (M.face_shift != nullptr && M.face_shift[f] != 0)) continue;
    const bool upwind = a.scheme == SWEEP_SCHEME_ALIGNED ? !isnan(wf[M.face_twin[f]])
                                                         : orient(ox, oy, oz, M.face_normal + 3 * f) < -a.eps;
    if (!upwind) continue;
    // nb is upwind of c: flag c in nb's row (or in its overflow list)
    int32_t* row = a.dnw + (U.task_base + nb) * W;
    for (int q = 0; q < W; ++q) {
      const int e = row[q];
      if (e == c) row[q] = c | kBigFlag;
      if (q == W - 1 && e < -1) {
        int32_t* ov = a.dn_ovf + (-(e + 2));
        for (int r = 1; r <= ov[0]; ++r)
          if (ov[r] == c) ov[r] = c | kBigFlag;
      }
    }
  }
}

constexpr int kFrontierCap = 2048;  // frontier entries kept in LDS per level

// Inclusive prefix sum over the 64 lanes of a wavefront (all lanes active):
// shifts of 1, 2, 4, 8 inside each row of 16 lanes, then the row totals are
// carried into the following rows with the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ int wave_inclusive_sum(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Kahn's algorithm for one (mesh, direction) unit per workgroup: tasks without
// upwind dependencies form level 0; solving a level decrements the counters of
// its tasks' downwind cells and those reaching zero form the next level.  The
// schedule lists every level's cells in the order they were appended (slots
// [lp[l], lp[l+1]) hold level l), together with its inverse.
// LDSCNT: the counters live in LDS as 4-bit fields; the value 15 marks a cell
// whose count (>= 15) is kept in global memory instead (it is never changed, so
// reading the field to pick the counter is race-free).
// NCH: chunks of 4 entries of a downwind row that are loaded at once (rows are
// -1 padded; NCH covers the longest list, or the whole row when some list
// continues in the overflow area).
template <bool LDSCNT, int NCH>
__global__ __launch_bounds__(kKahnBlock(NCH)) void k_kahn(DagBuildArgs a) {
  extern __shared__ uint32_t nib[];
  __shared__ int fr[2][kFrontierCap];
  __shared__ int s_cnt[3];
  const Unit U = a.units[blockIdx.x];
  const int C = U.n_cells;
  const int64_t tb = U.task_base;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63;
  int32_t* cnt = a.cnt + tb;
  // counters in global memory: one byte per cell, four to a word, so that the
  // counters of a whole unit (C bytes) stay in the last-level caches
  uint8_t* cnt8 = reinterpret_cast<uint8_t*>(cnt);
  uint32_t* cntw = reinterpret_cast<uint32_t*>(cnt);
  int32_t* sched = a.sched + tb;
  int32_t* spill = sched;  // frontier entries beyond the LDS copy (rewritten in place)
  int32_t* lp = a.lp + U.lp_base;
  const int W = a.dn_width;
  const int Wr4 = W / 4;  // chunks per row
  if (tid < 3) s_cnt[tid] = 0;
  const int nwords = (C + 7) / 8;  // counter words; 64 dummy words follow
  if (LDSCNT) {
    if (tid < 64) nib[nwords + tid] = 0u;
    for (int wi = tid; wi < nwords; wi += nthr) {
      int n[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) n[j] = a.indeg[tb + min(8 * wi + j, C - 1)];
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = 8 * wi + j;
        if (c < C) {
          if (n[j] >= 15) cnt[c] = n[j];
          v |= (uint32_t)min(n[j], 15) << (4 * j);
        }
      }
      nib[wi] = v;
    }
  }
  __syncthreads();
  // level 0: cells without upwind dependencies (global counters: the in-degrees
  // of kInitBatch cells per thread are loaded together, then stored as bytes)
  constexpr int kInitBatch = LDSCNT ? 1 : 8;
  for (int c0 = 0; c0 < C; c0 += kInitBatch * nthr) {
    int n[kInitBatch];
    if (!LDSCNT) {
#pragma unroll
      for (int j = 0; j < kInitBatch; ++j) {
        const int c = c0 + j * nthr + tid;
        n[j] = c < C ? a.indeg[tb + c] : -1;
      }
    }
#pragma unroll
    for (int j = 0; j < kInitBatch; ++j) {
      const int c = c0 + j * nthr + tid;
      bool ready = false;
      if (c < C) {
        if (LDSCNT) {
          ready = ((nib[c >> 3] >> (4 * (c & 7))) & 15u) == 0u;
        } else {
          cnt8[c] = (uint8_t)n[j];  // below 256 (the host checks the largest in-degree)
          ready = n[j] == 0;
        }
      }
      const unsigned long long m = __ballot(ready);
      if (m != 0ull) {
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&s_cnt[0], __popcll(m));
        base = __shfl(base, leader);
        if (ready) {
          const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
          if (slot < kFrontierCap) fr[0][slot] = c;
          else spill[slot] = c;
        }
      }
    }
  }
  __syncthreads();
  int head = 0;
  int tail = s_cnt[0];
  int l = 0;
  __syncthreads();
  if (tid == 0) {
    s_cnt[0] = 0;
    lp[0] = 0;
    lp[1] = tail;
  }
  __syncthreads();
  const int4* sent4 = reinterpret_cast<const int4*>(a.dnw + a.dn_sentinel);
  // The last wavefront makes every global store of the level loop (the
  // schedule and the level pointers; the inverse schedule is written when the
  // levels are sorted, k_sort_levels) and never waits for a load;
  // the other wavefronts process the frontier and only load, so their waits for
  // row loads never include a store (the vector-memory counter is in order).
  const int nwork = nthr - 64;
  const bool writer = tid >= nwork;
  // Level l: the frontier is [head, tail); its pushes count in s_cnt[l % 3].
  // s_cnt[(l + 1) % 3] was last read right after the barrier that ended level
  // l - 2, so it can be cleared now for level l + 1; one barrier per level.
  while (head < tail) {
    if (tid == 0) s_cnt[(l + 1) % 3] = 0;
    int* s_push = &s_cnt[l % 3];
    const int* frc = fr[l & 1];
    int* frn = fr[(l + 1) & 1];
    const bool fr_lds = tail - head <= kFrontierCap;  // the whole frontier is in LDS
    if (writer) {
      // the level's cells in slot order form the schedule (entries past the LDS
      // copy are in place already; each store is issued without waiting)
      const int n = min(tail - head, kFrontierCap);
      for (int i = lane; i < n; i += 64) sched[head + i] = frc[i];
      if (lane == 0) lp[l + 1] = tail;
    }
    for (int kb = head; !writer && kb < tail; kb += nwork) {
      const int k = kb + tid;
      const bool active = k < tail;
      if (__ballot(active) == 0ull) continue;  // wavefront without tasks this round
      const int kk = k - head;
      int c;
      if (fr_lds) {
        c = active ? frc[kk] : 0;
      } else {
        c = !active ? 0 : (kk < kFrontierCap ? frc[kk] : spill[k]);
        // no load of this path stays in flight: the common path's waits for the
        // loads of earlier levels are then counted exactly
        __builtin_amdgcn_s_waitcnt(0);
      }
      // all NCH chunk loads are unconditional: lanes without a task, and chunks
      // past the row width, read a sentinel row of -1 instead (an address
      // select), so they are in flight together
      const int4* row4 = active ? reinterpret_cast<const int4*>(a.dnw + (tb + c) * W) : sent4;
      int4 v[NCH];
#pragma unroll
      for (int q = 0; q < NCH; ++q) v[q] = (q < Wr4 ? row4 : sent4)[q];
      // a counter in global memory: 32-bit words of four byte counters (LDSCNT,
      // the counters of cells with 15 or more dependencies: whole words)
      auto dec_global = [&](int nb) -> bool {
        if (LDSCNT) {
          const int old = __hip_atomic_fetch_add(cnt + nb, -1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
          return old == 1;
        }
        const uint32_t sh = (uint32_t)(nb & 3) * 8u;
        const uint32_t old = __hip_atomic_fetch_add(cntw + (nb >> 2), 0u - (1u << sh), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
        return ((old >> sh) & 255u) == 1u;
      };
      uint32_t wm = 0;  // bit 4q+i: cell i of chunk q became ready
      if (LDSCNT) {
        // rows are -1 padded at the end, so the wavefront's non-empty chunks are
        // the first nq; inside them every entry issues one LDS decrement without
        // a branch (padding and flagged entries use the lane's private dummy
        // word and a zero operand); flagged entries (counters kept in global
        // memory) are decremented there afterwards
        int nq = 0;
#pragma unroll
        for (int q = 0; q < NCH; ++q) nq += __ballot(v[q].x >= 0) != 0ull ? 1 : 0;
        const int dummy = nwords + lane;
        uint32_t old[4 * NCH];
        bool any_big = false;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          if (q >= nq) break;
          const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = xs[i];
            const bool big = e >= 0 && (e & kBigFlag) != 0;
            const bool lds = e >= 0 && !big;
            any_big |= big;
            const uint32_t sh = (uint32_t)(e & 7) * 4u;
            old[4 * q + i] = atomicSub(&nib[lds ? e >> 3 : dummy], lds ? (1u << sh) : 0u);
          }
        }
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          if (q >= nq) break;
          const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = xs[i];
            const uint32_t sh = (uint32_t)(e & 7) * 4u;
            const bool ready = e >= 0 && (e & kBigFlag) == 0 && ((old[4 * q + i] >> sh) & 15u) == 1u;
            wm |= (uint32_t)ready << (4 * q + i);
          }
        }
        if (__ballot(any_big) != 0ull) {
#pragma unroll
          for (int q = 0; q < NCH; ++q) {
            if (q >= nq) break;
            const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (xs[i] >= 0 && (xs[i] & kBigFlag) != 0)
                wm |= (uint32_t)dec_global(xs[i] & ~kBigFlag) << (4 * q + i);
          }
        }
      } else {
        // counters in global memory: every real entry of the wavefront's
        // non-empty chunks issues its atomic before the first result is used;
        // padding lanes issue none (the memory system is the bottleneck here:
        // an atomic on a shared dummy word costs as much as a real one)
        int nq = 0;
#pragma unroll
        for (int q = 0; q < NCH; ++q) nq += __ballot(v[q].x >= 0) != 0ull ? 1 : 0;
        uint32_t old[4 * NCH];
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          if (q >= nq) break;
          const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int nb = xs[i] & ~kBigFlag;
            const uint32_t sh = (uint32_t)(nb & 3) * 8u;
            old[4 * q + i] = xs[i] >= 0 ? __hip_atomic_fetch_add(cntw + (nb >> 2), 0u - (1u << sh),
                                                                 __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_WORKGROUP)
                                        : 0u;
          }
        }
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          if (q >= nq) break;
          const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t sh = (uint32_t)(xs[i] & 3) * 8u;
            wm |= (uint32_t)(xs[i] >= 0 && ((old[4 * q + i] >> sh) & 255u) == 1u) << (4 * q + i);
          }
        }
      }
      // a full row may end in a pointer to its overflow list (rare): one
      // wavefront push per extra entry
      int ptr = -1;
#pragma unroll
      for (int q = 0; q < NCH; ++q) ptr = q == Wr4 - 1 ? v[q].w : ptr;
      if (__ballot(ptr < -1) != 0ull) {
        const int o = ptr < -1 ? -(ptr + 2) : 0;
        const int no = ptr < -1 ? a.dn_ovf[o] : 0;
        int mx = no;
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) mx = max(mx, __shfl_xor(mx, sh));
        for (int i = 0; i < mx; ++i) {
          const int e = i < no ? a.dn_ovf[o + 1 + i] : -1;
          const int nb = e >= 0 ? e & ~kBigFlag : -1;
          bool ready = false;
          if (nb >= 0) {
            const uint32_t sh = (uint32_t)(nb & 7) * 4u;
            if (LDSCNT && (e & kBigFlag) == 0) {
              const uint32_t old = atomicSub(&nib[nb >> 3], 1u << sh);
              ready = ((old >> sh) & 15u) == 1u;
            } else {
              ready = dec_global(nb);
            }
          }
          const unsigned long long m = __ballot(ready);
          if (m != 0ull) {
            const int leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(s_push, __popcll(m));
            base = __shfl(base, leader);
            if (ready) {
              const int r = base + __popcll(m & ((1ull << lane) - 1ull));
              if (r < kFrontierCap) frn[r] = nb;
              else spill[tail + r] = nb;
            }
          }
        }
      }
      // ready cells: one wavefront prefix sum and one LDS atomic per wavefront
      const int n = __popc(wm);
      const int incl = wave_inclusive_sum(n);
      const int total = __builtin_amdgcn_readlane(incl, 63);
      if (total > 0) {
        int base = 0;
        if (lane == 63) base = atomicAdd(s_push, total);
        int r = __builtin_amdgcn_readlane(base, 63) + incl - n;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (wm & (1u << (4 * q + i))) {
              const int cell = xs[i] & ~kBigFlag;
              if (r < kFrontierCap) frn[r] = cell;
              else spill[tail + r] = cell;
              ++r;
            }
          }
        }
      }
    }
    __syncthreads();
    head = tail;
    tail += s_cnt[l % 3];
    ++l;
  }
  if (tid == 0) lp[l + 1] = tail;
  if (tid == 0) {
    a.depth[blockIdx.x] = l;
    if (tail != C) atomicOr(a.err, 1);
  }
}

// Every level's cells in ascending cell id (the canonical order, so the
// schedule no longer depends on the order Kahn's wavefronts appended them),
// and the inverse schedule.  Workgroup b of a unit sorts the unit's levels b,
// b + kSortPerUnit, ... in LDS (bitonic, padded to a power of two); a level
// wider than kSortCap keeps its order.  Consecutive tasks of a level then lie
// close in the spatially numbered cells, so the per-task gathers and the
// cell-order result stores of the later kernels share cache lines.
constexpr int kSortCap = 4096;
constexpr int kSortBlock = 256;
constexpr int kSortPerUnit = 16;  // workgroups per unit

__global__ __launch_bounds__(kSortBlock) void k_sort_levels(DagBuildArgs a) {
  __shared__ int key[kSortCap];
  const int u = blockIdx.x / kSortPerUnit;
  const Unit U = a.units[u];
  const int depth = a.depth[u];
  int32_t* sched = a.sched + U.task_base;
  int32_t* inv = a.inv + U.task_base;
  const int32_t* lp = a.lp + U.lp_base;
  for (int l = blockIdx.x % kSortPerUnit; l < depth; l += kSortPerUnit) {
    const int k0 = lp[l], n = lp[l + 1] - k0;
    if (n > kSortCap || n < 2) {
      for (int i = threadIdx.x; i < n; i += kSortBlock) inv[sched[k0 + i]] = k0 + i;
      continue;
    }
    int P = 2;
    while (P < n) P <<= 1;
    for (int i = threadIdx.x; i < P; i += kSortBlock) key[i] = i < n ? sched[k0 + i] : INT_MAX;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < P / 2; i += kSortBlock) {
          const int lo = 2 * i - (i & (stride - 1));  // pair (lo, lo + stride)
          const int hi = lo + stride;
          const bool up = (lo & size) == 0;
          const int x = key[lo], y = key[hi];
          if ((x > y) == up) {
            key[lo] = y;
            key[hi] = x;
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < n; i += kSortBlock) {
      const int c = key[i];
      sched[k0 + i] = c;
      inv[c] = k0 + i;
    }
    __syncthreads();  // the next level reuses the keys
  }
}

// Row lengths of every task at its schedule slot (the input of the row-pointer scan).
__global__ __launch_bounds__(kCountBlock) void k_gather_len(DagBuildArgs a) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int u = unit_of_block(a.blk_base, a.n_units, blk);
  const Unit U = a.units[u];
  const int k = (blk - a.blk_base[u]) * kCountBlock + threadIdx.x;
  if (k >= U.n_cells) return;
  const int64_t t = U.task_base + k;
  // slots past the scheduled tasks (a cyclic graph, reported after the build) get no row
  const int scheduled = a.lp[U.lp_base + a.depth[u]];
  const int c = k < scheduled ? a.sched[t] : -1;
  a.len_up[t] = c >= 0 ? a.indeg[U.task_base + c] : 0;
  a.len_dn[t] = c >= 0 ? a.rowlen_dn[U.task_base + c] : 0;
  a.aperp_s[t] = c >= 0 ? a.aperp[U.task_base + c] : 0.0f;
  a.vol_s[t] = c >= 0 ? (float)a.meshes[U.mesh].cell_volume[c] : 0.0f;
}

// Per mesh: the largest face count of a cell, and the overflow room the wide
// rows need ((faces + 2) ints per direction for every cell with more than
// row_cap faces), accumulated into out[0] (max) and out[1] (sum).
__global__ __launch_bounds__(256) void k_face_stats(const int64_t* face_ptr, int n_cells, int row_cap, int n_dirs,
                             unsigned long long* out) {
  unsigned long long mx = 0, sum = 0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += gridDim.x * blockDim.x) {
    const unsigned long long nf = (unsigned long long)(face_ptr[c + 1] - face_ptr[c]);
    mx = nf > mx ? nf : mx;
    if (nf > (unsigned long long)row_cap) sum += (nf + 2) * (unsigned long long)n_dirs;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long m2 = __shfl_xor(mx, o);
    mx = m2 > mx ? m2 : mx;
    sum += __shfl_xor(sum, o);
  }
  // one atomic pair per block: same-address atomics from every wave serialise
  __shared__ unsigned long long part[2][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][w] = mx;
    part[1][w] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      mx = part[0][i] > mx ? part[0][i] : mx;
      sum += part[1][i];
    }
    atomicMax(out, mx);
    atomicAdd(out + 1, sum);
  }
}

// Per face: the neighbour code (>= 0: interior neighbour, -1: vacuum wall,
// -(nb + 2): periodic image of cell nb), which the row fill reads next to the
// face's signed weight instead of the FP64 geometry.
__global__ void k_face_codes(MeshDev M, int32_t* fcode) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= M.n_faces) return;
  const int nb = M.face_nbr[f];
  const bool periodic = M.face_shift != nullptr && M.face_shift[f] != 0;
  fcode[f] = nb < 0 ? -1 : (periodic ? -(nb + 2) : nb);
}

// Rows of the upwind and downwind lists, which lie in schedule order; the
// tasks are visited in cell order: each wavefront takes 64 consecutive cells
// of one unit, so that the face records it reads are contiguous and the
// neighbours' schedule positions (from the unit's inverse schedule) are
// gathered from a few lines.  Every lane first loads one cell's task (schedule
// slot, row pointers, face range); then, 16 cells per round, 16 lanes share
// one task, one face per lane, 16 faces at a time.  Each face's neighbour code
// and signed weight (from k_count) give its class; a ballot over the 16 lanes
// gives every entry its place in the row (rows keep the cell's face order).
// Cells of one level that are consecutive in id have consecutive slots, so
// their rows are written next to each other.
constexpr int kFillBlock = 256;

// Five wavefronts per SIMD: the register budget (at most 102 VGPRs) still
// compiles without spills.
template <bool ALIGNED>
__global__ __launch_bounds__(kFillBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_fill(DagBuildArgs a) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int u = unit_of_block(a.blk_base, a.n_units, blk);
  const Unit U = a.units[u];
  const MeshDev M = a.meshes[U.mesh];
  const int64_t tb = U.task_base;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int32_t* inv = a.inv + tb;
  const float* wf = a.wface + (int64_t)a.D * M.face_off + (int64_t)U.dir * M.n_faces;
  const int kw = (blk - a.blk_base[u]) * kFillBlock + (threadIdx.x & ~63);
  if (kw >= U.n_cells) return;
  // lane L: the task of cell kw + L (cells left out of the schedule of a cyclic
  // graph, reported after the build, have slot -1 and get no row)
  const int cl = kw + lane;
  const int k = cl < U.n_cells ? inv[cl] : -1;
  const bool kv = k >= 0 && k < a.lp[U.lp_base + a.depth[u]];
  const int kc = kv ? k : 0;
  const int c = kv ? cl : 0;
  const int64_t eu0 = a.up_ptr[tb + kc];
  const int64_t ed0 = a.dn_ptr[tb + kc];
  const int64_t f0 = M.face_ptr[c];
  const int nf = kv ? (int)(M.face_ptr[c + 1] - f0) : 0;
  const int rounds = min(4, (U.n_cells - kw + 15) >> 4);
  const uint32_t below = (1u << li) - 1u;
  for (int r = 0; r < rounds; ++r) {
    // group g handles slots kw + 16 r + 4 g + j, j = 0..3
    int64_t eu[4], ed[4], fb[4];
    int nfj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int src = 16 * r + 4 * g + j;
      eu[j] = __shfl(eu0, src);
      ed[j] = __shfl(ed0, src);
      fb[j] = __shfl(f0, src);
      nfj[j] = __shfl(nf, src);
    }
    int mx = max(max(nfj[0], nfj[1]), max(nfj[2], nfj[3]));
    mx = max(mx, __shfl_xor(mx, 16));
    mx = max(mx, __shfl_xor(mx, 32));
    for (int h = 0; h * 16 < mx; ++h) {
      const int fo = h * 16 + li;
      int code[4];
      float ws[4], wi[4];  // the face's own signed weight; scheme (b): its twin's
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t f = fo < nfj[j] ? fb[j] + fo : 0;  // face 0 exists
        code[j] = M.fcode[f];
        ws[j] = wf[f];
        if (ALIGNED) wi[j] = wf[code[j] != -1 ? M.face_twin[f] : f];
      }
      int pos[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) pos[j] = inv[code[j] >= 0 ? code[j] : 0];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bool up, dn;
        float w, wu;
        if (ALIGNED) {
          // radiation leaves through the faces the cell chose and enters through
          // the faces whose twin the neighbour chose
          up = fo < nfj[j] && code[j] >= 0 && !isnan(wi[j]);
          dn = fo < nfj[j] && code[j] >= 0 && !isnan(ws[j]);
          w = ws[j];
          wu = wi[j];
        } else {
          const bool has = fo < nfj[j] && !isnan(ws[j]);
          const bool in = has && signbit(ws[j]);
          up = in && code[j] >= 0;           // interior inflow
          dn = has && !in && code[j] >= 0;   // interior outflow
          w = wu = fabsf(ws[j]);
        }
        const uint32_t mu = (uint32_t)(__ballot(up) >> (16 * g)) & 0xffffu;
        const uint32_t md = (uint32_t)(__ballot(dn) >> (16 * g)) & 0xffffu;
        if (up) a.up[eu[j] + __popc(mu & below)] = make_int2(pos[j], __float_as_int(wu));
        if (dn) a.dn[ed[j] + __popc(md & below)] = make_int2(pos[j], __float_as_int(w));
        eu[j] += __popc(mu);
        ed[j] += __popc(md);
      }
    }
  }
}

// Periodic half-faces of every cell of mesh M (neighbour code -(nb + 2)).
__global__ void k_pcount(DagBuildArgs a, MeshDev M) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M.n_cells) return;
  int n = 0;
  for (int64_t f = M.face_ptr[c]; f < M.face_ptr[c + 1]; ++f) n += M.fcode[f] < -1 ? 1 : 0;
  a.npf[M.cell_off + c] = n;
  a.pflag[M.cell_off + c] = n > 0 ? 1 : 0;
}

// The periodic cells of mesh M in cell order with their periodic half-faces in
// face order (the face and its partner).
__global__ void k_plist(DagBuildArgs a, MeshDev M) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M.n_cells) return;
  const int gc = M.cell_off + c;
  const int64_t pc = a.pc_off[gc];
  const bool per = a.pc_off[gc + 1] > pc;
  a.pc_map[gc] = per ? (int)pc : -1;
  if (!per) return;
  a.pcell[pc] = gc;
  a.pf_ptr[pc] = (int32_t)a.pf_off[gc];
  int64_t j = a.pf_off[gc];
  for (int64_t f = M.face_ptr[c]; f < M.face_ptr[c + 1]; ++f) {
    const int code = M.fcode[f];
    if (code >= -1) continue;
    a.pface[j] = (int32_t)f;
    a.pnb[j] = M.cell_off + (-(code + 2));
    ++j;
  }
}

// Per (direction, periodic cell of mesh M): the inflow and outflow weight of
// each periodic half-face (the classes and weights k_fill gives the row
// entries, 0 where the half-face carries nothing that way) and the cell's task.
__global__ void k_pdir(DagBuildArgs a, MeshDev M, int mesh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.D * a.n_pc) return;
  const int pc = (int)(i % a.n_pc);
  const int d = (int)(i / a.n_pc);
  const int c = a.pcell[pc] - M.cell_off;
  if (c < 0 || c >= M.n_cells) return;  // a cell of another mesh
  const float* wf = a.wface + (int64_t)a.D * M.face_off + (int64_t)d * M.n_faces;
  for (int j = a.pf_ptr[pc]; j < a.pf_ptr[pc + 1]; ++j) {
    const int f = a.pface[j];
    float fw, aw;
    if (a.scheme == SWEEP_SCHEME_ALIGNED) {
      // inflow: the neighbour's share through the twin; outflow: the cell's own
      const float wi = wf[M.face_twin[f]];
      const float ws = wf[f];
      fw = isnan(wi) ? 0.0f : wi;
      aw = isnan(ws) ? 0.0f : ws;
    } else {
      const float ws = wf[f];
      const bool has = !isnan(ws);
      const bool in = has && signbit(ws);
      fw = in ? fabsf(ws) : 0.0f;
      aw = has && !in ? fabsf(ws) : 0.0f;
    }
    a.pwf[(int64_t)d * a.n_pf + j] = fw;
    a.pwa[(int64_t)d * a.n_pf + j] = aw;
  }
  const Unit U = a.units[mesh * a.D + d];
  a.ptask[i] = (int32_t)(U.task_base + a.inv[U.task_base + c]);
}

// First row entry of every level (per unit), so a level's rows form one block.
__global__ void k_level_entries(DagBuildArgs a) {
  const Unit U = a.units[blockIdx.x];
  const int depth = a.depth[blockIdx.x];
  for (int l = threadIdx.x; l <= depth + 1; l += blockDim.x) {
    const int64_t k = U.task_base + a.lp[U.lp_base + l];
    a.lev_up[U.lp_base + l] = a.up_ptr[k];
    a.lev_dn[U.lp_base + l] = a.dn_ptr[k];
  }
}

__global__ void k_unit_entries(const Unit* units, int32_t n_units, const int64_t* up_ptr,
                               const int64_t* dn_ptr, int64_t* out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_units) return;
  const int64_t t0 = units[u].task_base, t1 = t0 + units[u].n_cells;
  out[2 * u] = up_ptr[t1] - up_ptr[t0];
  out[2 * u + 1] = dn_ptr[t1] - dn_ptr[t0];
}

// Tasks per level, one workgroup per unit.
__global__ void k_level_widths(const Unit* units, const int32_t* lp, int32_t mesh,
                               unsigned long long* width, int32_t n_levels) {
  const Unit U = units[blockIdx.x];
  if (mesh >= 0 && U.mesh != mesh) return;
  const int32_t* l = lp + U.lp_base;
  for (int k = threadIdx.x; k < min(U.depth, n_levels); k += blockDim.x)
    atomicAdd(width + k, (unsigned long long)(l[k + 1] - l[k]));
}

// Steps of the level-synchronous sweep, one workgroup per unit: every level l
// (w tasks, e the larger of its upwind and downwind row entries) is cut into
// n = max(1, ceil(w / cap_t), ceil(1.15 e / cap_e)) runs of consecutive
// schedule positions with equal task counts (floor(c w / n) from the level's
// start).  The tasks of a run are independent, so each run is one step of the
// sweep; the 15 % margin keeps the runs' entry counts within cap_e for rows of
// ordinary spread (a run above it is still correct, on the sweep's slower
// path).  Writes the steps' first positions and entries (plus one closing
// step) from step_base[u], and their number.
constexpr int kStepsBlock = 256;
__global__ __launch_bounds__(kStepsBlock) void k_steps(const Unit* units, const int32_t* lp,
                                                       const int64_t* lev_up, const int64_t* lev_dn,
                                                       const int64_t* up_ptr, const int64_t* dn_ptr,
                                                       const int64_t* step_base, int32_t cap_t,
                                                       int32_t cap_e, int32_t* sk, int64_t* seu,
                                                       int64_t* sed, int32_t* n_steps) {
  __shared__ int s_scan[kStepsBlock];
  __shared__ int s_carry;
  const Unit U = units[blockIdx.x];
  const int tid = threadIdx.x;
  const int32_t* l = lp + U.lp_base;
  const int64_t* lu = lev_up + U.lp_base;
  const int64_t* ld = lev_dn + U.lp_base;
  const int64_t base = step_base[blockIdx.x];
  const int64_t cap = step_base[blockIdx.x + 1] - base;  // room for the steps and the closing one
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int l0 = 0; l0 < U.depth; l0 += kStepsBlock) {
    const int lv = l0 + tid;
    int n = 0, k0 = 0, w = 0;
    if (lv < U.depth) {
      k0 = l[lv];
      w = l[lv + 1] - k0;
      const int64_t e = max(lu[lv + 1] - lu[lv], ld[lv + 1] - ld[lv]);
      const int64_t ne = (e * 115 + 100LL * cap_e - 1) / (100LL * cap_e);
      n = max(1, max((w + cap_t - 1) / cap_t, (int)ne));
    }
    s_scan[tid] = n;
    __syncthreads();
    for (int o = 1; o < kStepsBlock; o <<= 1) {  // inclusive scan over the block
      const int x = tid >= o ? s_scan[tid - o] : 0;
      __syncthreads();
      s_scan[tid] += x;
      __syncthreads();
    }
    const int off = s_carry + s_scan[tid] - n;
    // (the host sizes the table above every count; a count past it is reported)
    for (int c = 0; c < n && off + c + 1 < cap; ++c) {
      const int kk = k0 + (int)(((int64_t)c * w) / n);
      sk[base + off + c] = kk;
      seu[base + off + c] = up_ptr[U.task_base + kk];
      sed[base + off + c] = dn_ptr[U.task_base + kk];
    }
    __syncthreads();
    if (tid == kStepsBlock - 1) s_carry += s_scan[tid];
    __syncthreads();
  }
  if (tid == 0) {
    const int ns = s_carry;
    if (ns + 1 > cap) {
      n_steps[blockIdx.x] = -1;
      return;
    }
    sk[base + ns] = U.n_cells;
    seu[base + ns] = up_ptr[U.task_base + U.n_cells];
    sed[base + ns] = dn_ptr[U.task_base + U.n_cells];
    n_steps[blockIdx.x] = ns;
  }
}

__global__ void k_d2f(const double* in, float* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned grid1d(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// LDS of k_count: the face tile, then (when it fits) one downwind row per thread.
size_t count_lds_bytes(int max_faces, int dn_width) {
  (void)max_faces;
  return tile_lds_bytes();
}

hipError_t launch_count(const DagBuildArgs& a, int32_t n_cblocks, int32_t lds_limit, hipStream_t s) {
  if (n_cblocks <= 0) return hipSuccess;
  if (a.scheme == SWEEP_SCHEME_ALIGNED) {
    const size_t tile = tile_lds_bytes();
    hipError_t e = hipFuncSetAttribute((const void*)k_count_aligned,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)tile);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_aligned, dim3(n_cblocks), dim3(kCountThreads), tile, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // upwind counts once every cell's choice is written
    hipLaunchKernelGGL(k_count_in, dim3(n_cblocks), dim3(kCountThreads), 0, s, a);
    return hipGetLastError();
  }
  const size_t tile = tile_lds_bytes();
  const size_t staged = tile + (size_t)kCountThreads * a.dn_width * 4;
  const bool stage = staged <= (size_t)lds_limit - 64;
  const size_t lds = stage ? staged : tile;
  const void* fn = stage ? (const void*)k_count<true> : (const void*)k_count<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (stage) hipLaunchKernelGGL(k_count<true>, dim3(n_cblocks), dim3(kCountThreads), lds, s, a);
  else hipLaunchKernelGGL(k_count<false>, dim3(n_cblocks), dim3(kCountThreads), lds, s, a);
  return hipGetLastError();
}

template <int NCH>
hipError_t launch_kahn_n(const DagBuildArgs& a, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_kahn<true, NCH>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_kahn<true, NCH>), dim3(a.n_units), dim3(kKahnBlock(NCH)), lds, s, a);
  return hipGetLastError();
}

template <int NCH>
hipError_t launch_kahn_g(const DagBuildArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_kahn<false, NCH>), dim3(a.n_units), dim3(kKahnBlock(NCH)), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_kahn(const DagBuildArgs& a, bool lds_counters, int32_t max_cells, hipStream_t s) {
  if (lds_counters) {
    const size_t lds = sizeof(uint32_t) * (size_t)((max_cells + 7) / 8 + 64);
    switch (a.dn_chunks) {
      case 0: case 1: case 2: case 3: case 4: return launch_kahn_n<4>(a, lds, s);
      case 5: return launch_kahn_n<5>(a, lds, s);
      case 6: return launch_kahn_n<6>(a, lds, s);
      case 7: return launch_kahn_n<7>(a, lds, s);
      default: return launch_kahn_n<8>(a, lds, s);
    }
  }
  switch (a.dn_chunks) {
    case 0: case 1: case 2: case 3: case 4: return launch_kahn_g<4>(a, s);
    default: return launch_kahn_g<8>(a, s);
  }
}

hipError_t launch_mark(const DagBuildArgs& a, int32_t n_big, hipStream_t s) {
  if (n_big <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark, dim3((n_big + 63) / 64), dim3(64), 0, s, a, n_big);
  return hipGetLastError();
}

hipError_t launch_sort_levels(const DagBuildArgs& a, hipStream_t s) {
  if (a.n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_levels, dim3(a.n_units * kSortPerUnit), dim3(kSortBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_len(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_len, dim3(n_blocks), dim3(kCountBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  if (a.scheme == SWEEP_SCHEME_ALIGNED)
    hipLaunchKernelGGL(k_fill<true>, dim3(n_blocks), dim3(kFillBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_fill<false>, dim3(n_blocks), dim3(kFillBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pcount(const DagBuildArgs& a, const MeshDev& m, hipStream_t s) {
  if (m.n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pcount, dim3(grid1d(m.n_cells, 256)), dim3(256), 0, s, a, m);
  return hipGetLastError();
}

hipError_t launch_plist(const DagBuildArgs& a, const MeshDev& m, hipStream_t s) {
  if (m.n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plist, dim3(grid1d(m.n_cells, 256)), dim3(256), 0, s, a, m);
  return hipGetLastError();
}

hipError_t launch_pdir(const DagBuildArgs& a, const MeshDev& m, int32_t mesh, hipStream_t s) {
  const int64_t n = (int64_t)a.D * a.n_pc;
  if (m.n_cells <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pdir, dim3(grid1d(n, 256)), dim3(256), 0, s, a, m, mesh);
  return hipGetLastError();
}

hipError_t launch_face_stats(const int64_t* face_ptr, int32_t n_cells, int32_t row_cap, int32_t n_dirs,
                             unsigned long long* out, hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(256, grid1d(n_cells, 256));
  hipLaunchKernelGGL(k_face_stats, dim3(grid), dim3(256), 0, s, face_ptr, n_cells, row_cap, n_dirs, out);
  return hipGetLastError();
}

hipError_t launch_face_codes(const MeshDev& m, int32_t* fcode, hipStream_t s) {
  if (m.n_faces <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_codes, dim3(grid1d(m.n_faces, 256)), dim3(256), 0, s, m, fcode);
  return hipGetLastError();
}

hipError_t launch_level_entries(const DagBuildArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_level_entries, dim3(a.n_units), dim3(256), 0, s, a);
  return hipGetLastError();
}

struct WidenToI64 {
  __host__ __device__ int64_t operator()(int32_t v) const { return (int64_t)v; }
};

hipError_t launch_scan_len(const int32_t* in, int64_t* out, int64_t n, void* tmp, size_t* tmp_bytes,
                           hipStream_t s) {
  // exclusive prefix sum of int32 row lengths into int64 row pointers (the
  // lengths are widened as they are read, so the sums never overflow);
  // tmp == nullptr queries the temporary storage size
  hipcub::TransformInputIterator<int64_t, WidenToI64, const int32_t*> it(in, WidenToI64());
  return hipcub::DeviceScan::ExclusiveSum(tmp, *tmp_bytes, it, out, (int)n, s);
}

hipError_t launch_unit_entries(const Unit* units, int32_t n_units, const int64_t* up_ptr,
                               const int64_t* dn_ptr, int64_t* out, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_entries, dim3(grid1d(n_units, 256)), dim3(256), 0, s, units, n_units,
                     up_ptr, dn_ptr, out);
  return hipGetLastError();
}

hipError_t launch_level_widths(const Unit* units, int32_t n_units, const int32_t* lp, int32_t mesh,
                               int64_t* width, int32_t n_levels, hipStream_t s) {
  if (n_units <= 0 || n_levels <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_widths, dim3(n_units), dim3(256), 0, s, units, lp, mesh,
                     reinterpret_cast<unsigned long long*>(width), n_levels);
  return hipGetLastError();
}

hipError_t launch_steps(const Unit* units, int32_t n_units, const int32_t* lp, const int64_t* lev_up,
                        const int64_t* lev_dn, const int64_t* up_ptr, const int64_t* dn_ptr,
                        const int64_t* step_base, int32_t cap_t, int32_t cap_e, int32_t* step_k,
                        int64_t* step_eu, int64_t* step_ed, int32_t* n_steps, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_steps, dim3(n_units), dim3(kStepsBlock), 0, s, units, lp, lev_up, lev_dn,
                     up_ptr, dn_ptr, step_base, cap_t, cap_e, step_k, step_eu, step_ed, n_steps);
  return hipGetLastError();
}

hipError_t launch_d2f(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_d2f, dim3(grid1d(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid1d(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace sweep
