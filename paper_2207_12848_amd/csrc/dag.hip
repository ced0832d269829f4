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
//             stored in schedule order so a level's rows are contiguous
#include <hipcub/hipcub.hpp>

#include <type_traits>

#include "internal.h"

namespace sweep {

namespace {

constexpr int kCountBlock = 256;
constexpr int kTileCells = 32;  // cells per tile of the cell-order kernels
constexpr int kKahnBlock = 512;

__device__ __forceinline__ double orient(double ox, double oy, double oz, const double* n) {
  const double a = ox * n[0];
  const double b = oy * n[1];
  const double c = oz * n[2];
  return (a + b) + c;
}

// Unit of block b (units own consecutive block ranges).
__device__ __forceinline__ int unit_of_block(const int32_t* blk_base, int n_units, int b) {
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk_base[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The cell-order kernels stage a tile of kTileCells consecutive cells' faces
// in LDS with coalesced loads; the workgroup then covers every direction, 32
// consecutive lanes handling the tile's cells for one direction.
struct FaceTile {
  int c0, cend;       // cells [c0, cend) of mesh m
  int64_t f0;         // first face of the tile
  const int64_t* fp;  // LDS copy of face_ptr[c0 .. cend] (relative to f0)
  const double* nrm;
  const double* area;
  const int32_t* nbr;
  const int8_t* shift;
};

__device__ __forceinline__ FaceTile stage_tile(const DagBuildArgs& a, const MeshDev& M, int c0,
                                               unsigned char* smem, int max_faces) {
  FaceTile T;
  T.c0 = c0;
  T.cend = min(c0 + kTileCells, M.n_cells);
  const int nc = T.cend - c0;
  T.f0 = M.face_ptr[c0];
  const int nf = (int)(M.face_ptr[T.cend] - T.f0);
  const int cap = kTileCells * max_faces;
  int64_t* fp = reinterpret_cast<int64_t*>(smem);
  double* nrm = reinterpret_cast<double*>(fp + kTileCells + 1);
  double* area = nrm + 3 * cap;
  int32_t* nbr = reinterpret_cast<int32_t*>(area + cap);
  int8_t* shift = reinterpret_cast<int8_t*>(nbr + cap);
  for (int i = threadIdx.x; i <= nc; i += blockDim.x) fp[i] = M.face_ptr[c0 + i] - T.f0;
  for (int i = threadIdx.x; i < 3 * nf; i += blockDim.x) nrm[i] = M.face_normal[3 * T.f0 + i];
  for (int i = threadIdx.x; i < nf; i += blockDim.x) {
    area[i] = M.face_area[T.f0 + i];
    nbr[i] = M.face_nbr[T.f0 + i];
    shift[i] = M.face_shift != nullptr ? M.face_shift[T.f0 + i] : (int8_t)0;
  }
  T.fp = fp;
  T.nrm = nrm;
  T.area = area;
  T.nbr = nbr;
  T.shift = shift;
  return T;
}

size_t tile_lds_bytes(int max_faces) {
  const size_t cap = (size_t)kTileCells * max_faces;
  return 8 * (kTileCells + 1) + cap * (24 + 8 + 4 + 1);
}

// Per task: upwind/downwind counts, Aperp = sum of outflow w, boundary outflow
// weights and the fixed-width list of downwind cells.
__global__ __launch_bounds__(kCountBlock) void k_count(DagBuildArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_max[2];
  if (threadIdx.x < 2) s_max[threadIdx.x] = 0;
  const int m = a.cblk_mesh[blockIdx.x];
  const MeshDev M = a.meshes[m];
  const FaceTile T = stage_tile(a, M, a.cblk_c0[blockIdx.x], smem, a.max_faces);
  __syncthreads();
  const int ci = threadIdx.x % kTileCells;
  const int c = T.c0 + ci;
  const int W = a.dn_width;
  int mi = 0, mo = 0;
  if (c < T.cend) {
    const int fb = (int)T.fp[ci], fe = (int)T.fp[ci + 1];
    for (int d = threadIdx.x / kTileCells; d < a.D; d += kCountBlock / kTileCells) {
      const double ox = a.dirs[3 * d], oy = a.dirs[3 * d + 1], oz = a.dirs[3 * d + 2];
      const int64_t t = a.units[m * a.D + d].task_base + c;
      int nup = 0, npin = 0, ndn = 0;
      double ap = 0.0, wall = 0.0, per = 0.0;
      int32_t* row = a.dnw + t * W;
      for (int f = fb; f < fe; ++f) {
        const double sv = orient(ox, oy, oz, T.nrm + 3 * f);
        const int nb = T.nbr[f];
        const bool periodic = T.shift[f] != 0;
        if (sv > a.eps) {
          const double w = T.area[f] * fabs(sv);
          ap += w;
          if (nb < 0) wall += w;
          else if (periodic) per += w;
          else row[ndn++] = nb;
        } else if (sv < -a.eps && nb >= 0) {
          if (periodic) ++npin; else ++nup;
        }
      }
      for (int q = ndn; q < W; ++q) row[q] = -1;
      a.indeg[t] = nup;
      a.rowlen_up[t] = nup + npin;
      a.rowlen_dn[t] = ndn;
      a.aperp[t] = (float)ap;
      a.bnd[t] = make_float2((float)wall, (float)per);
      mi = max(mi, nup);
      mo = max(mo, ndn);
    }
  }
  atomicMax(&s_max[0], mi);
  atomicMax(&s_max[1], mo);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(a.stats, s_max[0]);
    atomicMax(a.stats + 1, s_max[1]);
  }
}

constexpr int kFrontierCap = 2048;  // frontier entries mirrored in LDS per level
constexpr int kRowChunks = 8;       // downwind-row chunks (4 cells each) loaded at once

// Append `cell` to the schedule if `want`, one LDS atomic per wavefront; the
// new level's first kFrontierCap entries are mirrored in LDS.
__device__ __forceinline__ void push_ready(bool want, int cell, int* s_tail, int32_t* sched,
                                           int32_t* inv, int* fr_next, int next_base) {
  const unsigned long long m = __ballot(want);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(s_tail, __popcll(m));
  base = __shfl(base, leader);
  if (want) {
    const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
    sched[slot] = cell;
    inv[cell] = slot;
    if (slot - next_base < kFrontierCap) fr_next[slot - next_base] = cell;
  }
}

// Kahn's algorithm for one (mesh, direction) unit per workgroup: tasks without
// upwind dependencies form level 0; solving a level decrements the counters of
// its tasks' downwind cells and those reaching zero form the next level.
// LDSCNT: the counters live in LDS as 4-bit fields; the value 15 marks a cell
// whose count (>= 15) is kept in global memory instead (it is never changed, so
// reading the field to pick the counter is race-free).
template <bool LDSCNT>
__global__ __launch_bounds__(kKahnBlock) void k_kahn(DagBuildArgs a) {
  extern __shared__ uint32_t nib[];
  __shared__ int fr[2][kFrontierCap];
  __shared__ int s_tail;
  const Unit U = a.units[blockIdx.x];
  const int C = U.n_cells;
  const int64_t tb = U.task_base;
  const int tid = threadIdx.x, nthr = blockDim.x;
  int32_t* cnt = a.cnt + tb;
  int32_t* sched = a.sched + tb;
  int32_t* inv = a.inv + tb;
  int32_t* level = a.level + tb;
  int32_t* lp = a.lp + U.lp_base;
  const int W = a.dn_width;
  if (tid == 0) s_tail = 0;
  if (LDSCNT) {
    for (int wi = tid; wi < (C + 7) / 8; wi += nthr) {
      uint32_t v = 0;
      for (int j = 0; j < 8; ++j) {
        const int c = 8 * wi + j;
        if (c < C) {
          const int n = a.indeg[tb + c];
          if (n >= 15) cnt[c] = n;
          v |= (uint32_t)min(n, 15) << (4 * j);
        }
      }
      nib[wi] = v;
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < C; c0 += nthr) {
    const int c = c0 + tid;
    bool ready = false;
    if (c < C) {
      const int n = a.indeg[tb + c];
      if (!LDSCNT) cnt[c] = n;
      ready = (n == 0);
    }
    push_ready(ready, c, &s_tail, sched, inv, fr[0], 0);
  }
  __syncthreads();
  int head = 0;
  int tail = s_tail;
  int l = 0;
  if (tid == 0) {
    lp[0] = 0;
    lp[1] = tail;
  }
  while (head < tail) {
    const int* frc = fr[l & 1];
    int* frn = fr[(l + 1) & 1];
    // a level whose frontier fits the LDS copy reads it from LDS only (no
    // vector-memory load joins the path, so nothing waits on older stores)
    auto level_body = [&](auto from_lds) {
      constexpr bool FROM_LDS = decltype(from_lds)::value;
      // wave-uniform rounds: lanes without a task take part with nothing to push
      for (int kb = head; kb < tail; kb += nthr) {
        const int k = kb + tid;
        const bool active = k < tail;
        if (__ballot(active) == 0ull) continue;  // wavefront without tasks this round
        const int c = !active ? 0 : (FROM_LDS ? frc[k - head] : sched[k]);
        if (active) level[c] = l;
        // the whole downwind row is loaded at once (W is a multiple of 4), every
        // counter is decremented, then the ready cells are compacted with one
        // wavefront prefix sum
        // every chunk load is unconditional: lanes without a task, and chunks past
      // the row width, read a sentinel row of -1 instead (an address select), so
      // all loads are in flight together
      const int4* sent4 = reinterpret_cast<const int4*>(a.dnw + a.dn_sentinel);
      const int4* row4 = active ? reinterpret_cast<const int4*>(a.dnw + (tb + c) * W) : sent4;
        const int W4 = W >> 2;
        int4 v[kRowChunks];
  #pragma unroll
        for (int q = 0; q < kRowChunks; ++q) v[q] = (q < W4 ? row4 : sent4)[q];
        auto dec_global = [&](int nb) -> bool {
          const int old = __hip_atomic_fetch_add(cnt + nb, -1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
          return old == 1;
        };
        uint32_t wm = 0;  // bit 4q+i: cell i of chunk q became ready
        if (LDSCNT) {
          // batched: every counter word is read, then every LDS decrement issued,
          // so each batch costs two LDS round trips
          uint32_t word[4 * kRowChunks];
  #pragma unroll
          for (int q = 0; q < kRowChunks; ++q) {
            const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
  #pragma unroll
            for (int i = 0; i < 4; ++i) word[4 * q + i] = nib[(xs[i] >= 0 ? xs[i] : 0) >> 3];
          }
          uint32_t old[4 * kRowChunks];
  #pragma unroll
          for (int q = 0; q < kRowChunks; ++q) {
            const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int nb = xs[i];
              const uint32_t sh = (uint32_t)(nb & 7) * 4u;
              old[4 * q + i] = 0;
              if (nb >= 0 && ((word[4 * q + i] >> sh) & 15u) != 15u)
                old[4 * q + i] = atomicSub(&nib[nb >> 3], 1u << sh);
            }
          }
  #pragma unroll
          for (int q = 0; q < kRowChunks; ++q) {
            const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int nb = xs[i];
              if (nb < 0) continue;
              const uint32_t sh = (uint32_t)(nb & 7) * 4u;
              bool ready;
              if (((word[4 * q + i] >> sh) & 15u) != 15u) ready = ((old[4 * q + i] >> sh) & 15u) == 1u;
              else ready = dec_global(nb);
              wm |= (uint32_t)ready << (4 * q + i);
            }
          }
        } else {
  #pragma unroll
          for (int q = 0; q < kRowChunks; ++q) {
            const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
  #pragma unroll
            for (int i = 0; i < 4; ++i)
              if (xs[i] >= 0) wm |= (uint32_t)dec_global(xs[i]) << (4 * q + i);
          }
        }
        auto dec = [&](int nb) -> bool {
          if (nb < 0) return false;
          const uint32_t sh = (uint32_t)(nb & 7) * 4u;
          if (LDSCNT && ((nib[nb >> 3] >> sh) & 15u) != 15u) {
            const uint32_t o = atomicSub(&nib[nb >> 3], 1u << sh);
            return ((o >> sh) & 15u) == 1u;
          }
          return dec_global(nb);
        };
        // rows wider than kRowChunks chunks (cells with more than 32 faces)
        for (int q = kRowChunks; q < W4; ++q) {
          const int4 x = row4[q];
          const int xs[4] = {x.x, x.y, x.z, x.w};
          for (int i = 0; i < 4; ++i) {
            const bool ready = dec(xs[i]);
            push_ready(ready, xs[i], &s_tail, sched, inv, frn, tail);
          }
        }
        // wavefront prefix sum of the ready counts, one LDS atomic per wavefront
        const int n = __popc(wm);
        const int lane = threadIdx.x & 63;
        int incl = n;
  #pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(incl, o);
          if (lane >= o) incl += y;
        }
        const unsigned long long act = __ballot(1);
        const int last = 63 - __clzll((long long)act);
        const int total = __shfl(incl, last);
        int base = 0;
        if (lane == last && total > 0) base = atomicAdd(&s_tail, total);
        base = __shfl(base, last) + incl - n;
  #pragma unroll
        for (int q = 0; q < kRowChunks; ++q) {
          const int xs[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (wm & (1u << (4 * q + i))) {
              const int slot = base++;
              sched[slot] = xs[i];
              inv[xs[i]] = slot;
              if (slot - tail < kFrontierCap) frn[slot - tail] = xs[i];
            }
          }
        }
      }
    };
    if (tail - head <= kFrontierCap) level_body(std::true_type{});
    else level_body(std::false_type{});
    __syncthreads();
    head = tail;
    tail = s_tail;
    ++l;
    if (tid == 0) lp[l + 1] = tail;
    __syncthreads();
  }
  if (tid == 0) {
    a.depth[blockIdx.x] = l;
    if (tail != C) atomicOr(a.err, 1);
  }
}

__global__ __launch_bounds__(kCountBlock) void k_gather_len(DagBuildArgs a) {
  const int u = unit_of_block(a.blk_base, a.n_units, blockIdx.x);
  const Unit U = a.units[u];
  const int k = (blockIdx.x - a.blk_base[u]) * kCountBlock + threadIdx.x;
  if (k >= U.n_cells) return;
  const int64_t t = U.task_base + k;
  const int c = a.sched[t];
  a.len_up[t] = a.rowlen_up[U.task_base + c];
  a.len_dn[t] = a.rowlen_dn[U.task_base + c];
}

// Rows of the upwind and downwind lists, written at the task's schedule
// position.  Entries follow the cell's face order, so the rows do not depend
// on the schedule.
__global__ __launch_bounds__(kCountBlock) void k_fill(DagBuildArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = a.cblk_mesh[blockIdx.x];
  const MeshDev M = a.meshes[m];
  const FaceTile T = stage_tile(a, M, a.cblk_c0[blockIdx.x], smem, a.max_faces);
  __syncthreads();
  const int ci = threadIdx.x % kTileCells;
  const int c = T.c0 + ci;
  if (c >= T.cend) return;
  const int fb = (int)T.fp[ci], fe = (int)T.fp[ci + 1];
  for (int d = threadIdx.x / kTileCells; d < a.D; d += kCountBlock / kTileCells) {
    const double ox = a.dirs[3 * d], oy = a.dirs[3 * d + 1], oz = a.dirs[3 * d + 2];
    const int64_t tb = a.units[m * a.D + d].task_base;
    const int32_t* inv = a.inv + tb;
    const int pos = inv[c];
    int64_t eu = a.up_ptr[tb + pos];
    int64_t ed = a.dn_ptr[tb + pos];
    for (int f = fb; f < fe; ++f) {
      const int nb = T.nbr[f];
      if (nb < 0) continue;
      const double sv = orient(ox, oy, oz, T.nrm + 3 * f);
      const bool periodic = T.shift[f] != 0;
      if (sv < -a.eps) {
        const float w = (float)(T.area[f] * fabs(sv));
        a.up[eu++] = make_int2(periodic ? -(nb + 1) : inv[nb], __float_as_int(w));
      } else if (sv > a.eps && !periodic) {
        const float w = (float)(T.area[f] * fabs(sv));
        a.dn[ed++] = make_int2(inv[nb], __float_as_int(w));
      }
    }
  }
}

// First row entry of every level (per unit), so a level's rows form one block.
__global__ void k_level_entries(DagBuildArgs a) {
  const Unit U = a.units[blockIdx.x];
  for (int l = threadIdx.x; l <= U.depth + 1; l += blockDim.x) {
    const int64_t k = U.task_base + a.lp[U.lp_base + l];
    a.lev_up[U.lp_base + l] = a.up_ptr[k];
    a.lev_dn[U.lp_base + l] = a.dn_ptr[k];
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

hipError_t launch_count(const DagBuildArgs& a, int32_t n_cblocks, hipStream_t s) {
  if (n_cblocks <= 0) return hipSuccess;
  const size_t lds = tile_lds_bytes(a.max_faces);
  hipError_t e = hipFuncSetAttribute((const void*)k_count, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_count, dim3(n_cblocks), dim3(kCountBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_kahn(const DagBuildArgs& a, bool lds_counters, int32_t max_cells, hipStream_t s) {
  if (lds_counters) {
    const size_t lds = sizeof(uint32_t) * (size_t)((max_cells + 7) / 8);
    hipError_t e = hipFuncSetAttribute((const void*)k_kahn<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kahn<true>, dim3(a.n_units), dim3(kKahnBlock), lds, s, a);
  } else {
    hipLaunchKernelGGL(k_kahn<false>, dim3(a.n_units), dim3(kKahnBlock), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_gather_len(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_len, dim3(n_blocks), dim3(kCountBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(const DagBuildArgs& a, int32_t n_cblocks, hipStream_t s) {
  if (n_cblocks <= 0) return hipSuccess;
  const size_t lds = tile_lds_bytes(a.max_faces);
  hipError_t e = hipFuncSetAttribute((const void*)k_fill, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill, dim3(n_cblocks), dim3(kCountBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_level_entries(const DagBuildArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_level_entries, dim3(a.n_units), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, size_t* tmp_bytes,
                           hipStream_t s) {
  // exclusive prefix sum; tmp == nullptr queries the temporary storage size
  return hipcub::DeviceScan::ExclusiveSum(tmp, *tmp_bytes, in, out, (int)n, s);
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
