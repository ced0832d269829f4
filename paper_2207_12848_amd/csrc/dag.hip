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

#include "internal.h"

namespace sweep {

namespace {

constexpr int kCountBlock = 256;
constexpr int kKahnBlock = 1024;

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

__global__ __launch_bounds__(kCountBlock) void k_count(DagBuildArgs a) {
  const int u = unit_of_block(a.blk_base, a.n_units, blockIdx.x);
  const Unit U = a.units[u];
  const int c = (blockIdx.x - a.blk_base[u]) * kCountBlock + threadIdx.x;
  if (c >= U.n_cells) return;
  const MeshDev M = a.meshes[U.mesh];
  const double ox = a.dirs[3 * U.dir], oy = a.dirs[3 * U.dir + 1], oz = a.dirs[3 * U.dir + 2];
  int nup = 0, npin = 0, ndn = 0;
  double aperp = 0.0, wall = 0.0, per = 0.0;
  for (int64_t f = M.face_ptr[c]; f < M.face_ptr[c + 1]; ++f) {
    const double s = orient(ox, oy, oz, M.face_normal + 3 * f);
    const int nb = M.face_nbr[f];
    const bool periodic = M.face_shift != nullptr && M.face_shift[f] != 0;
    if (s > a.eps) {
      const double w = M.face_area[f] * fabs(s);
      aperp += w;
      if (nb < 0) wall += w;
      else if (periodic) per += w;
      else ++ndn;
    } else if (s < -a.eps && nb >= 0) {
      if (periodic) ++npin; else ++nup;
    }
  }
  const int64_t t = U.task_base + c;
  a.indeg[t] = nup;
  a.rowlen_up[t] = nup + npin;
  a.rowlen_dn[t] = ndn;
  a.aperp[t] = (float)aperp;
  a.bnd[t] = make_float2((float)wall, (float)per);
}

// Append `cell` to the schedule if `want`, one LDS atomic per wavefront.
__device__ __forceinline__ void push_ready(bool want, int cell, int* s_tail, int32_t* sched,
                                           int32_t* inv) {
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
  }
}

__global__ __launch_bounds__(kKahnBlock) void k_kahn(DagBuildArgs a) {
  const Unit U = a.units[blockIdx.x];
  const MeshDev M = a.meshes[U.mesh];
  const int C = U.n_cells;
  const int64_t tb = U.task_base;
  int32_t* cnt = a.cnt + tb;
  int32_t* sched = a.sched + tb;
  int32_t* inv = a.inv + tb;
  int32_t* level = a.level + tb;
  int32_t* lp = a.lp + U.lp_base;
  const double ox = a.dirs[3 * U.dir], oy = a.dirs[3 * U.dir + 1], oz = a.dirs[3 * U.dir + 2];
  __shared__ int s_tail;
  if (threadIdx.x == 0) s_tail = 0;
  __syncthreads();
  // level 0: every task without upwind dependencies
  for (int c0 = 0; c0 < C; c0 += blockDim.x) {
    const int c = c0 + threadIdx.x;
    bool ready = false;
    if (c < C) {
      const int n = a.indeg[tb + c];
      cnt[c] = n;
      ready = (n == 0);
    }
    push_ready(ready, c, &s_tail, sched, inv);
  }
  __syncthreads();
  int head = 0;
  int tail = s_tail;
  int l = 0;
  if (threadIdx.x == 0) {
    lp[0] = 0;
    lp[1] = tail;
  }
  while (head < tail) {
    for (int k = head + threadIdx.x; k < tail; k += blockDim.x) {
      const int c = sched[k];
      level[c] = l;
      for (int64_t f = M.face_ptr[c]; f < M.face_ptr[c + 1]; ++f) {
        const int nb = M.face_nbr[f];
        bool want = false;
        if (nb >= 0 && !(M.face_shift != nullptr && M.face_shift[f] != 0) &&
            orient(ox, oy, oz, M.face_normal + 3 * f) > a.eps) {
          const int old = __hip_atomic_fetch_add(cnt + nb, -1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
          want = (old == 1);
        }
        push_ready(want, nb, &s_tail, sched, inv);
      }
    }
    __syncthreads();
    head = tail;
    tail = s_tail;
    ++l;
    if (threadIdx.x == 0) lp[l + 1] = tail;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
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

__global__ __launch_bounds__(kCountBlock) void k_fill(DagBuildArgs a) {
  const int u = unit_of_block(a.blk_base, a.n_units, blockIdx.x);
  const Unit U = a.units[u];
  const int k = (blockIdx.x - a.blk_base[u]) * kCountBlock + threadIdx.x;
  if (k >= U.n_cells) return;
  const MeshDev M = a.meshes[U.mesh];
  const double ox = a.dirs[3 * U.dir], oy = a.dirs[3 * U.dir + 1], oz = a.dirs[3 * U.dir + 2];
  const int64_t t = U.task_base + k;
  const int c = a.sched[t];
  const int32_t* inv = a.inv + U.task_base;
  int64_t eu = a.up_ptr[t];
  int64_t ed = a.dn_ptr[t];
  for (int64_t f = M.face_ptr[c]; f < M.face_ptr[c + 1]; ++f) {
    const int nb = M.face_nbr[f];
    if (nb < 0) continue;
    const double s = orient(ox, oy, oz, M.face_normal + 3 * f);
    const bool periodic = M.face_shift != nullptr && M.face_shift[f] != 0;
    if (s < -a.eps) {
      const float w = (float)(M.face_area[f] * fabs(s));
      a.up[eu++] = make_int2(periodic ? -(nb + 1) : inv[nb], __float_as_int(w));
    } else if (s > a.eps && !periodic) {
      const float w = (float)(M.face_area[f] * fabs(s));
      a.dn[ed++] = make_int2(inv[nb], __float_as_int(w));
    }
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

hipError_t launch_count(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3(n_blocks), dim3(kCountBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_kahn(const DagBuildArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_kahn, dim3(a.n_units), dim3(kKahnBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_len(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_len, dim3(n_blocks), dim3(kCountBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(n_blocks), dim3(kCountBlock), 0, s, a);
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
