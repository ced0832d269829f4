// Forward and adjoint sweep kernels and the per-cell reductions (gfx950).
//
// Schedule: one workgroup owns one (mesh, direction) sweep at a time and walks
// its levels in order (reverse order for the adjoint), one barrier per level.
// The tasks of a level are independent (their upwind tasks sit on earlier
// levels), so the workgroup's threads solve them in parallel; every task pulls
// its inflow from its upwind tasks' results in a fixed row order, so results do
// not depend on which thread runs which task.  Persistent form: a grid sized to
// the resident capacity takes (mesh, direction) units from an atomic counter,
// longest first.
//
// LDS ring: the results of the last `ring` tasks of the schedule are kept in
// LDS, indexed by schedule position modulo `ring`, so most upwind reads are LDS
// reads; an older upwind result is read back from global memory (it was stored
// at least one barrier earlier by the same workgroup).
#include "internal.h"

namespace sweep {

namespace {

constexpr float kInv4Pi = 0.0795774715459476678f;  // 1 / (4 pi)

template <int GN, bool REVERSE>
__global__ void k_sweep(SweepArgs a) {
  extern __shared__ float ring[];
  __shared__ int s_unit;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int R = a.ring_mask + 1;
  for (int it = 0;; ++it) {
    int ui;
    if (a.work_counter != nullptr) {
      if (tid == 0) s_unit = atomicAdd(a.work_counter, 1);
      __syncthreads();
      ui = s_unit;
      __syncthreads();
    } else {
      ui = it == 0 ? (int)blockIdx.x : a.n_units;
    }
    if (ui >= a.n_units) break;
    const Unit U = a.units[a.unit_order[ui]];
    const int64_t tb = U.task_base;
    const int32_t* sched = a.sched + tb;
    const int32_t* lp = a.lp + U.lp_base;
    const int64_t obase = ((int64_t)U.dir * a.C_total + U.cell_off) * a.G + a.g0;
    const int depth = U.depth;
    for (int step = 0; step < depth; ++step) {
      const int l = REVERSE ? depth - 1 - step : step;
      const int k0 = lp[l];
      const int k1 = lp[l + 1];
      for (int k = k0 + tid; k < k1; k += nthr) {
        const int c = sched[k];
        const int64_t e0 = a.row_ptr[tb + k];
        const int64_t e1 = a.row_ptr[tb + k + 1];
        double acc[GN];
        double pin[GN];
#pragma unroll
        for (int g = 0; g < GN; ++g) acc[g] = pin[g] = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
          const int2 en = a.ent[e];
          const double w = (double)__int_as_float(en.y);
          const int p = en.x;
          if (p >= 0) {
            const bool in_ring = REVERSE ? (p < k0 + R) : (p >= k1 - R);
            if (in_ring) {
              const float* r = ring + (p & a.ring_mask) * GN;
#pragma unroll
              for (int g = 0; g < GN; ++g) acc[g] += w * (double)r[g];
            } else {
              const float* q = a.out + obase + (int64_t)sched[p] * a.G;
#pragma unroll
              for (int g = 0; g < GN; ++g) acc[g] += w * (double)q[g];
            }
          } else if (a.phi_prev != nullptr) {
            const float* q = a.phi_prev + obase + (int64_t)(-p - 1) * a.G;
#pragma unroll
            for (int g = 0; g < GN; ++g) {
              const double v = w * (double)q[g];
              acc[g] += v;
              pin[g] += v;
            }
          }
        }
        const int64_t ci = (int64_t)(U.cell_off + c);
        const double V = (double)a.vol[ci];
        const double ap = (double)a.aperp[tb + c];
        float* r = ring + (k & a.ring_mask) * GN;
        float* o = a.out + obase + (int64_t)c * a.G;
#pragma unroll
        for (int g = 0; g < GN; ++g) {
          const int64_t cg = ci * a.G + a.g0 + g;
          const double kap = (double)a.kappa[cg];
          double s = (double)a.src[cg];
          if (!REVERSE) {
            if (a.jsum_prev != nullptr) s += (double)a.albedo * kap * V * (double)a.jsum_prev[cg];
            s *= (double)a.inv_D;
          }
          const float v = (float)((acc[g] + s) / (ap + kap * V));
          r[g] = v;
          o[g] = v;
        }
        if (!REVERSE && a.pin != nullptr) {
          float* pp = a.pin + obase + (int64_t)c * a.G;
#pragma unroll
          for (int g = 0; g < GN; ++g) pp[g] = (float)pin[g];
        }
      }
      __syncthreads();
    }
  }
}

template <bool REVERSE>
hipError_t launch_sweep_t(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                          int32_t ring, hipStream_t s) {
  const size_t lds = sweep_lds_bytes(gn, ring);
  switch (gn) {
    case 1: hipLaunchKernelGGL((k_sweep<1, REVERSE>), dim3(grid), dim3(block), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_sweep<2, REVERSE>), dim3(grid), dim3(block), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_sweep<3, REVERSE>), dim3(grid), dim3(block), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_sweep<4, REVERSE>), dim3(grid), dim3(block), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------- reductions
constexpr int kRedBlock = 256;
constexpr int kNPart = 9;

__global__ __launch_bounds__(kRedBlock) void k_reduce(ReduceArgs a) {
  __shared__ double part[kRedBlock][kNPart];
  const int m = a.blk_mesh[blockIdx.x];
  const int c0 = a.blk_cell0[blockIdx.x];
  const int G = a.G;
  const int i = threadIdx.x;
  const int c = c0 + i / G;
  const int g = i % G;
  const int mend = a.mesh_off[m] + a.mesh_cells[m];
  const bool active = (i < a.cells_per_block * G) && (c < mend);
  double v[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) v[k] = 0.0;
  if (active) {
    const int64_t cg = (int64_t)c * G + g;
    const int64_t stride = a.C_total * G;
    const int lc = c - a.mesh_off[m];
    double js = 0.0, pn = 0.0, esc = 0.0, pout = 0.0;
    for (int d = 0; d < a.D; ++d) {
      const double ph = (double)a.phi[d * stride + cg];
      js += ph;
      if (a.pin != nullptr) pn += (double)a.pin[d * stride + cg];
      if (a.last) {
        const float2 b = a.bnd[a.units[m * a.D + d].task_base + lc];
        esc += (double)b.x * ph;
        pout += (double)b.y * ph;
      }
    }
    if (a.pin_sum != nullptr) a.pin_sum[cg] = pn;
    if (a.last) {
      const double V = (double)a.vol[c];
      const double kap = (double)a.kappa[cg];
      const double ka = (1.0 - (double)a.albedo) * kap;
      const double ks = (double)a.albedo * kap;
      const double ab = ka * V * js;
      a.jsum[cg] = (float)js;
      a.J[cg] = (float)(js * (double)kInv4Pi);
      a.absorbed[cg] = (float)ab;
      const double jp = a.jsum_prev != nullptr ? (double)a.jsum_prev[cg] : 0.0;
      v[0] = (double)a.emission[cg];
      v[1] = ab;
      v[2] = esc;
      v[3] = pn;
      v[4] = pout;
      v[5] = ks * V * (jp - js);
      if (a.pin_prev != nullptr) {
        const double po = a.pin_prev[cg];
        const double den = pn + po;
        v[6] = den > 0.0 ? fabs(pn - po) / den : 0.0;
        v[7] = fabs(pn - po);
        v[8] = den;
      }
    }
  }
  if (!a.last) return;
#pragma unroll
  for (int k = 0; k < kNPart; ++k) part[i][k] = v[k];
  __syncthreads();
  if (i < G) {
    double s[kNPart];
#pragma unroll
    for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
    for (int j = i; j < kRedBlock; j += G) {
#pragma unroll
      for (int k = 0; k < kNPart; ++k) {
        if (k == 6) s[k] = fmax(s[k], part[j][k]);
        else s[k] += part[j][k];
      }
    }
#pragma unroll
    for (int k = 0; k < kNPart; ++k) a.partial[((int64_t)blockIdx.x * G + i) * kNPart + k] = s[k];
  }
}

__global__ void k_totals(const double* partial, const int32_t* mesh_blk_base, int32_t n_meshes,
                         int32_t G, double* totals) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_meshes * G) return;
  const int m = t / G, g = t % G;
  double s[kNPart];
  for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
  for (int b = mesh_blk_base[m]; b < mesh_blk_base[m + 1]; ++b)
    for (int k = 0; k < kNPart; ++k) {
      const double x = partial[((int64_t)b * G + g) * kNPart + k];
      if (k == 6) s[k] = fmax(s[k], x); else s[k] += x;
    }
  double* o = totals + (int64_t)t * 8;
  for (int k = 0; k < 7; ++k) o[k] = s[k];
  o[7] = s[8] > 0.0 ? s[7] / s[8] : 0.0;
}

__global__ void k_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t n,
                           float* gsrc, double* dk, double* de) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double V = (double)vol[i / G];
  const double ga = (double)dA[i];
  const double ka = (1.0 - (double)albedo) * (double)kappa[i];
  gsrc[i] = (float)((double)dJ[i] * (double)kInv4Pi + ga * ka * V);
  dk[i] = ga * (1.0 - (double)albedo) * V * (double)jsum_last[i];
  de[i] = 0.0;
}

__global__ void k_adj_reduce(AdjReduceArgs a, double* dk, double* de) {
  const int64_t n = a.C_total * a.G;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ls = 0.0, lph = 0.0;
  for (int d = 0; d < a.D; ++d) {
    const double l = (double)a.lam[d * n + i];
    ls += l;
    lph += l * (double)a.phi[d * n + i];
  }
  const double V = (double)a.vol[i / a.G];
  const double prev = a.jsum_prev != nullptr ? (double)a.jsum_prev[i] : 0.0;
  const double alb = (double)a.albedo;
  const double invD = (double)a.inv_D;
  dk[i] += -V * lph + alb * V * ls * prev * invD;
  de[i] += ls * invD;
  a.gsrc_next[i] = (float)(alb * (double)a.kappa[i] * V * ls * invD);
}

__global__ void k_d2f_pair(const double* a, const double* b, float* oa, float* ob, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    oa[i] = (float)a[i];
    ob[i] = (float)b[i];
  }
}

inline unsigned grid1d(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t sweep_lds_bytes(int32_t gn, int32_t ring) { return (size_t)gn * ring * sizeof(float); }

hipError_t launch_sweep_fwd(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            int32_t ring, hipStream_t s) {
  return launch_sweep_t<false>(a, gn, grid, block, ring, s);
}

hipError_t launch_sweep_adj(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            int32_t ring, hipStream_t s) {
  return launch_sweep_t<true>(a, gn, grid, block, ring, s);
}

hipError_t set_sweep_lds_limit(int32_t bytes) {
  const void* fns[] = {(const void*)k_sweep<1, false>, (const void*)k_sweep<2, false>,
                       (const void*)k_sweep<3, false>, (const void*)k_sweep<4, false>,
                       (const void*)k_sweep<1, true>,  (const void*)k_sweep<2, true>,
                       (const void*)k_sweep<3, true>,  (const void*)k_sweep<4, true>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reduce(const ReduceArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(n_blocks), dim3(kRedBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_totals(const double* partial, const int32_t* mesh_blk_base, int32_t n_meshes,
                         int32_t G, double* totals, hipStream_t s) {
  const int n = n_meshes * G;
  hipLaunchKernelGGL(k_totals, dim3(grid1d(n, 64)), dim3(64), 0, s, partial, mesh_blk_base,
                     n_meshes, G, totals);
  return hipGetLastError();
}

hipError_t launch_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t C,
                           float* gsrc, double* dk, double* de, hipStream_t s) {
  const int64_t n = C * G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_init, dim3(grid1d(n, 256)), dim3(256), 0, s, dJ, dA, kappa, vol,
                     jsum_last, albedo, G, n, gsrc, dk, de);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const AdjReduceArgs& a, double* dk, double* de, hipStream_t s) {
  const int64_t n = a.C_total * a.G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_reduce, dim3(grid1d(n, 256)), dim3(256), 0, s, a, dk, de);
  return hipGetLastError();
}

hipError_t launch_d2f_pair(const double* a, const double* b, float* oa, float* ob, int64_t n,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_d2f_pair, dim3(grid1d(n, 256)), dim3(256), 0, s, a, b, oa, ob, n);
  return hipGetLastError();
}

}  // namespace sweep
