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
// reads; an older upwind result is prefetched from global memory a step ahead
// (it was stored at least two barriers earlier by the same workgroup).
#include <float.h>

#include "internal.h"
#include "sweep.h"

namespace sweep {

namespace {

constexpr float kInv4Pi = 0.0795774715459476678f;  // 1 / (4 pi)

// Buffer loads: every per-unit array is addressed through a buffer resource
// (base in scalar registers, 32-bit offsets); offsets past the end read 0.
constexpr int32_t kBufFlags = 0x00020000;  // raw buffer, 32-bit data (gfx9 family)
constexpr uint32_t kOob = 0x7ffffff0u;     // an offset past the end of any buffer here

template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const T* p, int64_t bytes) {
  // the arguments are uniform; read from the first lane so that the descriptor
  // is built in scalar registers (a descriptor in vector registers costs a
  // loop over the distinct values at every access)
  const uint64_t a = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const int n = __builtin_amdgcn_readfirstlane((int)(p == nullptr ? 0 : bytes));
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, n,
                                           kBufFlags);
}

// Cache policy of the accesses the sweep makes once per step and never again
// (row entries, task records, results in cell order): non-temporal, so the L2
// keeps the schedule-order results that later steps read back.
constexpr int kStream = 2;

template <int POL = 0>
__device__ __forceinline__ int2 ld_b64(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(int2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, POL));
}
template <int POL = 0>
__device__ __forceinline__ int4 ld_b128(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, POL));
}
template <int POL = 0>
__device__ __forceinline__ int ld_b32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, POL);
}
__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __int_as_float(ld_b32(r, vo, so));
}
template <int POL = 0>
__device__ __forceinline__ void st_f32(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, (int)vo, 0, POL);
}

// GN consecutive FP32 values at byte offset vo + so of a buffer (one access for
// GN = 2 or 4; offsets past the buffer's end read zeros and drop stores).
template <int GN, int POL = 0>
__device__ __forceinline__ void ld_gn(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float* v) {
  if constexpr (GN == 4) {
    const int4 x = __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, POL));
    v[0] = __int_as_float(x.x);
    v[1] = __int_as_float(x.y);
    v[2] = __int_as_float(x.z);
    v[3] = __int_as_float(x.w);
  } else if constexpr (GN == 2) {
    const int2 x = __builtin_bit_cast(int2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, POL));
    v[0] = __int_as_float(x.x);
    v[1] = __int_as_float(x.y);
  } else {
#pragma unroll
    for (int g = 0; g < GN; ++g) v[g] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)(vo + 4u * g), (int)so, POL));
  }
}

template <int GN, int POL = 0>
__device__ __forceinline__ void st_gn(const float* v, __amdgpu_buffer_rsrc_t r, uint32_t vo) {
  if constexpr (GN == 4) {
    const int4 x = make_int4(__float_as_int(v[0]), __float_as_int(v[1]), __float_as_int(v[2]),
                             __float_as_int(v[3]));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) int, x), r, (int)vo, 0, POL);
  } else if constexpr (GN == 2) {
    const int2 x = make_int2(__float_as_int(v[0]), __float_as_int(v[1]));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) int, x), r, (int)vo, 0, POL);
  } else {
#pragma unroll
    for (int g = 0; g < GN; ++g) st_f32<POL>(v[g], r, vo + 4u * g);
  }
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The unit's buffers (uniform over the workgroup).
struct UnitBufs {
  __amdgpu_buffer_rsrc_t ent;    // row entries of the unit (from its first entry)
  __amdgpu_buffer_rsrc_t sched;  // schedule of the unit
  __amdgpu_buffer_rsrc_t rp;     // row pointers of the unit (int64)
  __amdgpu_buffer_rsrc_t den;    // [slot][G] at group g0 of the unit's first task
  __amdgpu_buffer_rsrc_t src;
  __amdgpu_buffer_rsrc_t outs;   // out_s at group g0 of the unit's first task: [slot][G]
  __amdgpu_buffer_rsrc_t out;    // out of this direction at group g0: [cell][G]
  int64_t ue0;                   // first row entry of the unit
};

// Record of one task: cell, row [r0, r1) relative to its step's first entry,
// denominator and source per group.
template <int GN>
struct TaskRec {
  int c;
  int r0, r1;
  float den[GN];
  float src[GN];
};

// Per-step values, uniform over the workgroup.
struct LevelInfo {
  int k0, k1;     // the step's task range (schedule positions)
  int ne;         // row entries of the step
  int nst;        // entries of the step held in LDS staging
  int64_t e0;     // first row entry of the step
};

// Entries of a staged row hold the LDS byte address of their value instead of a
// schedule position (the ring slot of a result inside the window, or the slot
// the older value was prefetched into) and their factor.  An entry whose value
// is not in LDS names the zero slot and marks its step for the global-memory
// path.

// Loads in flight for one step: the thread's share of the step's row block
// (raw entries, two per load) and the record of the thread's task of the step,
// with the step's bounds.  Lanes past the step read past the buffers' ends (no
// memory traffic, value 0).
template <int GN, int CH>
struct Pref {
  LevelInfo L;
  int4 st[CH / 2];
  int c;
  // low words of the row pointers of the task and the next one (two loads: a
  // register a load writes and nothing reads would be reused while the load is
  // in flight, and the wait for it would stall the next solve)
  int rp0, rp1;
  float den[GN];
  float src[GN];
};

template <int GN>
__device__ __forceinline__ void load_rec(const SweepArgs& a, const UnitBufs& B, int k, int64_t e0,
                                         TaskRec<GN>& t) {
  t.c = ld_b32(B.sched, 4u * (uint32_t)k, 0);
  t.r0 = (int)((uint32_t)ld_b32(B.rp, 8u * (uint32_t)k, 0) - (uint32_t)e0);
  t.r1 = (int)((uint32_t)ld_b32(B.rp, 8u * (uint32_t)(k + 1), 0) - (uint32_t)e0);
  ld_gn<GN>(B.den, 4u * (uint32_t)(k * a.G), 0, t.den);
  ld_gn<GN>(B.src, 4u * (uint32_t)(k * a.G), 0, t.src);
}

// Every thread issues the same loads at every step (fixed count, so the waits
// for the loads in flight stay exact); the offsets of lanes past the step are
// moved past the buffers' ends.  Entry pair i of thread t is entries
// 2 (t + i nthr) and 2 (t + i nthr) + 1 of the step's block.
template <int GN, int CH>
__device__ __forceinline__ void issue_pref(const SweepArgs& a, const UnitBufs& B, int tid, int nthr,
                                           Pref<GN, CH>& P) {
  const LevelInfo& L = P.L;
  const uint32_t eoff = 8u * (uint32_t)(L.e0 - B.ue0);
#pragma unroll
  for (int i = 0; i < CH / 2; ++i) {
    const int idx = 2 * (tid + i * nthr);
    P.st[i] = ld_b128<kStream>(B.ent, idx < L.nst ? 8u * (uint32_t)idx : kOob, eoff);
  }
  const bool act = L.k0 + tid < L.k1;
  const uint32_t k0 = (uint32_t)L.k0;
  P.c = ld_b32<kStream>(B.sched, act ? 4u * (uint32_t)tid : kOob, 4u * k0);
  P.rp0 = ld_b32<kStream>(B.rp, act ? 8u * (uint32_t)tid : kOob, 8u * k0);
  P.rp1 = ld_b32<kStream>(B.rp, act ? 8u * (uint32_t)tid + 8u : kOob, 8u * k0);
  const uint32_t vo = act ? 4u * (uint32_t)(tid * a.G) : kOob, so = 4u * k0 * (uint32_t)a.G;
  ld_gn<GN, kStream>(B.den, vo, so, P.den);
  ld_gn<GN, kStream>(B.src, vo, so, P.src);
}

// Inflow of one task per group.
template <int GN>
struct Inflow {
  float acc[GN];
};

// Schedule positions whose results are in the LDS ring while a step is solved,
// [lo, lo + n) with lo >= 0: forward, the last R positions up to the step's end;
// adjoint (steps in reverse order), the R positions from the step's start.
// The step's own writes never evict an upwind result inside the window.
struct Window {
  int lo;
  uint32_t n;
  __device__ __forceinline__ bool has(int p) const { return (uint32_t)(p - lo) < n; }
};

template <bool REVERSE>
__device__ __forceinline__ Window window(int k0, int k1, int R) {
  Window w;
  if (REVERSE) {
    w.lo = k0;
    w.n = (uint32_t)R;
  } else {
    w.lo = k1 - R > 0 ? k1 - R : 0;
    w.n = (uint32_t)(k1 - w.lo);
  }
  return w;
}

template <int GN>
__device__ __forceinline__ void finish_task(const SweepArgs& a, const UnitBufs& B,
                                            const TaskRec<GN>& t, int k, const Inflow<GN>& in,
                                            float* ring) {
  float* rr = ring + (k & a.ring_mask) * GN;
  const uint32_t oc = 4u * (uint32_t)(t.c * a.G), ok = 4u * (uint32_t)(k * a.G);
  float v[GN];
#pragma unroll
  for (int g = 0; g < GN; ++g) {
    v[g] = __fdiv_rn(__fadd_rn(in.acc[g], t.src[g]), t.den[g]);
    rr[g] = v[g];
  }
  st_gn<GN, kStream>(v, B.out, oc);
  st_gn<GN>(v, B.outs, ok);
}

// The common step: at most one task per thread and every inflow in LDS.  Every
// memory operation is issued unconditionally (a thread without a task writes
// the sink slot and stores past the buffers' ends, which are dropped), so each
// step issues a fixed number of vector-memory operations.
template <int GN>
__device__ __forceinline__ void finish_fast(const SweepArgs& a, const UnitBufs& B,
                                            const TaskRec<GN>& t, int k, const Inflow<GN>& in,
                                            float* ring, float* sink) {
  const bool act = t.c >= 0;
  float* rr = act ? ring + (k & a.ring_mask) * GN : sink;
  const uint32_t oc = act ? 4u * (uint32_t)(t.c * a.G) : kOob;
  const uint32_t ok = act ? 4u * (uint32_t)(k * a.G) : kOob;
  float v[GN];
#pragma unroll
  for (int g = 0; g < GN; ++g) {
    v[g] = __fdiv_rn(__fadd_rn(in.acc[g], t.src[g]), t.den[g]);
    rr[g] = v[g];
  }
  st_gn<GN, kStream>(v, B.out, oc);
  st_gn<GN>(v, B.outs, ok);
}

// GN consecutive groups of one task from a [slot][G] array (one load; offsets
// past the buffer's end read zeros without memory traffic).
template <int GN>
__device__ __forceinline__ void ld_groups(__amdgpu_buffer_rsrc_t r, uint32_t off, float* v) {
  if constexpr (GN == 4) {
    const int4 x = ld_b128(r, off, 0);
    v[0] = __int_as_float(x.x);
    v[1] = __int_as_float(x.y);
    v[2] = __int_as_float(x.z);
    v[3] = __int_as_float(x.w);
  } else if constexpr (GN == 2) {
    const int2 x = ld_b64(r, off, 0);
    v[0] = __int_as_float(x.x);
    v[1] = __int_as_float(x.y);
  } else {
#pragma unroll
    for (int g = 0; g < GN; ++g) v[g] = ld_f32(r, off + 4u * g, 0);
  }
}

// Inflow of one task in row order, in batches of 8 entries (the row's entries
// from the LDS staging buffer, or from global memory for levels that were not
// staged).  An entry inside the window reads its ring slot; an older result is
// loaded from out_s (stored at least one barrier earlier by this workgroup).
// Every load of a batch is issued before the first is used, so a batch
// costs one memory round trip whatever its mix.  The sum is the same sequence
// of fused multiply-adds in row order on every path; entries past the row's end
// (the rest of the batch) are skipped.
template <int GN, bool STAGED>
__device__ __forceinline__ Inflow<GN> gather(const SweepArgs& a, const UnitBufs& B,
                                             const TaskRec<GN>& t, const int2* stg, uint32_t eoff,
                                             const float* ring, Window w) {
  Inflow<GN> in;
#pragma unroll
  for (int g = 0; g < GN; ++g) in.acc[g] = 0.0f;
  for (int rb = t.r0; rb < t.r1; rb += 8) {
    int2 en[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      en[q] = STAGED ? stg[rb + q] : ld_b64(B.ent, 8u * (uint32_t)(rb + q), eoff);
    const int nr = t.r1 - rb;  // entries of the row in this batch
    float gv[8][GN], rv[8][GN];
    bool inw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = en[q].x;
      const bool val = q < nr;
      inw[q] = w.has(p);
      const bool glob = val && !inw[q];
      ld_groups<GN>(B.outs, glob ? 4u * (uint32_t)(p * a.G) : kOob, gv[q]);
      const float* v = ring + (p & a.ring_mask) * GN;
#pragma unroll
      for (int g = 0; g < GN; ++g) rv[q][g] = v[g];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool val = q < nr;
      const float y = __int_as_float(en[q].y);
#pragma unroll
      for (int g = 0; g < GN; ++g) {
        const float x = inw[q] ? rv[q][g] : gv[q][g];
        in.acc[g] = val ? __builtin_fmaf(y, x, in.acc[g]) : in.acc[g];
      }
    }
  }
  return in;
}

// Inflow of one task from its staged row, every value from LDS (`lds`: the base
// the entries' addresses are relative to), in batches of 8 with the same
// sequence of fused multiply-adds in row order as gather().  The entries of a
// batch past the row's end (the next row's, or padding naming the zero slot)
// take factor 0; adding +-0 x (x finite) leaves a sum that starts at +0 and only
// grows unchanged, so the result is gather()'s bit for bit.
template <int GN>
__device__ __forceinline__ Inflow<GN> gather_lds(const TaskRec<GN>& t, const int2* stg,
                                                 const unsigned char* lds) {
  Inflow<GN> in;
#pragma unroll
  for (int g = 0; g < GN; ++g) in.acc[g] = 0.0f;
  for (int rb = t.r0; rb < t.r1; rb += 8) {
    int2 en[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) en[q] = stg[rb + q];
    const int nr = t.r1 - rb;
    float rv[8][GN], y[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      y[q] = q < nr ? __int_as_float(en[q].y) : 0.0f;
      // value slots are GN floats at a multiple of GN floats: one LDS read
      const unsigned char* v = lds + en[q].x;
      if constexpr (GN == 4) {
        const float4 x = *reinterpret_cast<const float4*>(v);
        rv[q][0] = x.x;
        rv[q][1] = x.y;
        rv[q][2] = x.z;
        rv[q][3] = x.w;
      } else if constexpr (GN == 2) {
        const float2 x = *reinterpret_cast<const float2*>(v);
        rv[q][0] = x.x;
        rv[q][1] = x.y;
      } else {
#pragma unroll
        for (int g = 0; g < GN; ++g) rv[q][g] = reinterpret_cast<const float*>(v)[g];
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
      for (int g = 0; g < GN; ++g) in.acc[g] = __builtin_fmaf(y[q], rv[q][g], in.acc[g]);
    }
  }
  return in;
}

// One workgroup per (mesh, direction) unit at a time, steps in order (reverse
// for the adjoint), one barrier per step.  A step is a run of consecutive
// schedule positions inside one level (levels wider than the workgroup or
// with more entries than the staging buffer are cut into several), so its
// tasks are independent.  Each step's row block and each thread's task record
// are loaded NS - 1 steps ahead into registers (NS rotating sets).  Two steps
// ahead, the holder of each staged entry whose upwind result lies outside the
// LDS ring window loads that value from global memory; the step before it is solved the holder copies the value into the
// entry's own slot of the LDS value area and rewrites the entry to name its
// slot (ring slot or prefetched slot).  The solve then reads only LDS, and no
// load is waited for on the critical path of a common step.
// A value is prefetched only when it is final: at the prefetch (after the
// thread's solve of step t, for step t + 2) every step before t is complete,
// which covers every result outside the window when the ring holds at least
// three steps (R >= 3 x threads, as the host sizes it).
//
// LDS: [values: ring R slots | zero | sink | 2 x SE prefetched slots] x GN floats,
// then two staging buffers of SE + 8 entries.
// The rows hold graph edges only: the other pass's values through the periodic
// faces are folded into the sources before the launch.
template <int GN, bool REVERSE, int CH>
__global__ __launch_bounds__(kSweepMaxBlock(GN)) void k_sweep(SweepArgs a) {
  constexpr int NS = 3;
  extern __shared__ __align__(16) unsigned char smem[];
  float* vals = reinterpret_cast<float*>(smem);
  int2* stage = reinterpret_cast<int2*>(smem + a.stage_off);
  __shared__ int s_unit;
  // s_bad[b]: the running number of the last step staged in buffer b with an
  // entry whose value is not in LDS (such a step is solved from global memory)
  __shared__ int s_bad[2];
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int SE = CH * nthr;
  const int SP = SE + 8;  // staging buffer stride
  const int SMAX = SE - 8;  // entries staged per step; 8 padding entries follow them
  const int R = a.ring_mask + 1;
  const int zero = R;       // value slot that always holds zeros (padding entries)
  const int sink = R + 1;   // value slot the threads without a task write
  const int far0 = R + 2;   // prefetched slots of staging buffer b: far0 + b SE + entry index
  const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);  // the wavefront's first thread
  float* ring = vals;
  float* sinkp = vals + sink * GN;
  for (int i = tid; i < 2 * SP; i += nthr) stage[i] = make_int2(zero * GN * 4, 0);
  for (int i = tid; i < (R + 2 + 2 * SE) * GN; i += nthr) vals[i] = 0.0f;
  if (tid < 2) s_bad[tid] = -1;
  int gbase = 0;  // running number of this workgroup's step 0 of the current unit
  for (int it = 0;; ++it) {
    int ui;
    if (a.work_counter != nullptr) {
      if (tid == 0) s_unit = atomicAdd(a.work_counter, 1);
      __syncthreads();
      ui = __builtin_amdgcn_readfirstlane(s_unit);  // uniform: the unit's buffers stay scalar
      __syncthreads();
    } else {
      ui = it == 0 ? (int)blockIdx.x : a.n_units * a.n_chunks;
    }
    if (ui >= a.n_units * a.n_chunks) break;
    const int u = a.unit_order[ui / a.n_chunks];
    const int g0 = a.g0 + (ui % a.n_chunks) * GN;
    const Unit U = a.units[u];
    const int64_t tb = U.task_base;
    const int ns = a.n_steps[u];
    if (ns <= 0) continue;
    // step tables are read through the scalar cache (constant address space:
    // the sweep never writes them), so reading them never waits for the vector
    // loads in flight
    using cint = const __attribute__((address_space(4))) int32_t;
    using clong = const __attribute__((address_space(4))) int64_t;
    cint* SK = (cint*)(a.step_k + a.step_base[u]);
    clong* SEn = (clong*)(a.step_e + a.step_base[u]);
    const int64_t obase = ((int64_t)U.dir * a.C_total + U.cell_off) * a.G + g0;
    const int C = U.n_cells;
    UnitBufs B;
    {
      const int64_t ea = SEn[0], eb = SEn[ns];
      B.ue0 = ea < eb ? ea : eb;
      const int64_t ue1 = ea < eb ? eb : ea;
      B.ent = rsrc(a.ent + B.ue0, 8 * (ue1 - B.ue0));
    }
    B.sched = rsrc(a.sched + tb, 4 * (int64_t)C);
    B.rp = rsrc(a.row_ptr + tb, 8 * ((int64_t)C + 1));
    B.den = rsrc(a.tden + tb * a.G + g0, 4 * ((int64_t)C * a.G - g0));
    B.src = rsrc(a.tsrc + tb * a.G + g0, 4 * ((int64_t)C * a.G - g0));
    B.outs = rsrc(a.out_s + tb * a.G + g0, 4 * ((int64_t)C * a.G - g0));
    B.out = rsrc(a.out + obase, 4 * ((int64_t)C * a.G - g0));
    // step solved at iteration s (iterations past the last one repeat it: their
    // loads are issued and never used)
    auto info = [&](int s) -> LevelInfo {
      s = s < ns - 1 ? s : ns - 1;
      const int st = REVERSE ? ns - 1 - s : s;
      LevelInfo L;
      // the values are uniform: keep them in scalar registers
      L.k0 = __builtin_amdgcn_readfirstlane(SK[st]);
      L.k1 = __builtin_amdgcn_readfirstlane(SK[st + 1]);
      L.e0 = uniform64(SEn[st]);
      L.ne = (int)(uniform64(SEn[st + 1]) - L.e0);
      L.nst = L.ne < SMAX ? L.ne : SMAX;
      return L;
    };
    Pref<GN, CH> P[NS];
    float F[CH][GN];  // prefetched values of the thread's staged entries
    TaskRec<GN> cur;
    LevelInfo curL;
    // results final at the last prefetch: forward, positions below vis; adjoint,
    // positions from vis up
    int vis = REVERSE ? 0x7fffffff : 0, visF = vis;
    auto prefetchable = [&](int p, const Window& w, int v) -> bool {
      return !w.has(p) && (REVERSE ? p >= v : p < v);
    };
    auto issue = [&](int s, Pref<GN, CH>& Q) {
      Q.L = info(s);
      issue_pref<GN, CH>(a, B, tid, nthr, Q);
    };
    // the older results of the thread's staged entries of step s (one load per
    // entry; the others read past the buffer's end)
    auto farload = [&](const Pref<GN, CH>& Q) {
      const LevelInfo& L = Q.L;
      const Window w = window<REVERSE>(L.k0, L.k1, R);
      uint32_t po = 0;  // per entry: an older result to load
#pragma unroll
      for (int i = 0; i < CH / 2; ++i) {
        if (2 * (wbase + i * nthr) >= L.nst) continue;  // no entry of this wavefront
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int idx = 2 * (tid + i * nthr) + h;
          const int p = h ? Q.st[i].z : Q.st[i].x;
          po |= (uint32_t)(idx < L.nst && prefetchable(p, w, vis)) << (2 * i + h);
        }
      }
      // the loads of a wavefront whose lanes need none are not issued
      if (__ballot(po != 0u) != 0ull) {
#pragma unroll
        for (int i = 0; i < CH / 2; ++i)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int p = h ? Q.st[i].z : Q.st[i].x;
            ld_groups<GN>(B.outs, (po >> (2 * i + h)) & 1u ? 4u * (uint32_t)(p * a.G) : kOob,
                          F[2 * i + h]);
          }
      }
      visF = vis;
    };
    // staged entries of step s (value slots, followed by 8 padding entries that
    // name the zero slot with factor 0) and the prefetched values into the staging
    // buffer and value slots of s's parity; the thread's record into `cur`
    auto publish = [&](int s, const Pref<GN, CH>& Q) {
      const LevelInfo& L = Q.L;
      const int b = s & 1;
      int2* dst = stage + b * SP;
      const Window w = window<REVERSE>(L.k0, L.k1, R);
#pragma unroll
      for (int i = 0; i < CH / 2; ++i) {
        const int idx0 = 2 * (tid + i * nthr);
        int4 v = Q.st[i];
        if (2 * (wbase + i * nthr) >= L.nst + 8) {
          // no entry of this wavefront in the step: the registers loaded for it
          // (entries and prefetched values) are only consumed (a load nothing
          // reads would leave its wait to a later reuse of the registers)
          asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int g = 0; g < GN; ++g) asm volatile("" ::"v"(F[2 * i + h][g]));
          continue;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int idx = idx0 + h;
          const int p = h ? v.z : v.x;
          const bool val = idx < L.nst;
          const bool pf = val && prefetchable(p, w, visF);
          const int fs = far0 + b * SE + idx;
          const bool inw = w.has(p);
          const int slot = !val ? zero : (inw ? (p & a.ring_mask) : (pf ? fs : zero));
          if (val && !inw && !pf) s_bad[b] = gbase + s;
          if (pf) {
#pragma unroll
            for (int g = 0; g < GN; ++g) vals[fs * GN + g] = F[2 * i + h][g];
          }
          const int addr = slot * (GN * 4);
          if (h) {
            v.z = addr;
            v.w = !val ? 0 : v.w;
          } else {
            v.x = addr;
            v.y = !val ? 0 : v.y;
          }
        }
        if (idx0 < L.nst + 8) *reinterpret_cast<int4*>(dst + idx0) = v;
      }
      curL = L;
      const bool act = L.k0 + tid < L.k1;
      cur.c = act ? Q.c : -1;
      cur.r0 = act ? (int)((uint32_t)Q.rp0 - (uint32_t)L.e0) : 0;
      cur.r1 = act ? (int)((uint32_t)Q.rp1 - (uint32_t)L.e0) : 0;
#pragma unroll
      for (int g = 0; g < GN; ++g) {
        cur.den[g] = Q.den[g];
        cur.src[g] = Q.src[g];
      }
    };
    auto solve = [&](int s) {
      const int k0 = curL.k0, k1 = curL.k1;
      const int64_t e0 = curL.e0;
      const int2* stg = stage + (s & 1) * SP;
      const Window w = window<REVERSE>(k0, k1, R);
      const uint32_t eoff = 8u * (uint32_t)(e0 - B.ue0);
      vis = REVERSE ? k1 : k0;
      const bool bad = __builtin_amdgcn_readfirstlane(s_bad[s & 1]) == gbase + s;
      if (curL.nst == curL.ne && k1 - k0 <= nthr && !bad) {
        const Inflow<GN> in = gather_lds<GN>(cur, stg, smem);
        finish_fast<GN>(a, B, cur, k0 + tid, in, ring, sinkp);
        return;
      }
      for (int k = k0 + tid; k < k1; k += nthr) {
        TaskRec<GN> t;
        if (k == k0 + tid) t = cur; else load_rec<GN>(a, B, k, e0, t);
        const Inflow<GN> in = gather<GN, false>(a, B, t, nullptr, eoff, ring, w);
        finish_task<GN>(a, B, t, k, in, ring);
      }
      // the uncommon steps leave no memory operation of theirs in flight, so the
      // waits of the common steps are counted exactly
      __builtin_amdgcn_s_waitcnt(0);
    };
    // prologue: steps 0 .. NS - 1 in flight, the values of steps 0 and 1
    // prefetched, step 0 staged.  Iteration s then solves step s, stages step
    // s + 1 (its values were prefetched an iteration earlier), issues the loads
    // of step s + NS into the set it freed and prefetches the values of step
    // s + 2.
#pragma unroll
    for (int j = 0; j < NS; ++j) issue(j, P[j]);
    farload(P[0]);
    publish(0, P[0]);
    farload(P[1]);
    __syncthreads();
    for (int s = 0; s < ns; s += NS) {
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        if (s + j >= ns) break;
        solve(s + j);
        // unconditional (past the last step it stages a copy of the last step
        // into the staging buffer no solve reads), so every set of loads is
        // consumed on every path and the waits stay exact
        publish(s + j + 1, P[(j + 1) % NS]);
        issue(s + j + NS, P[j]);
        farload(P[(j + 2) % NS]);
        __syncthreads();
      }
    }
    gbase += ns + 1;  // past the last step's number and the one staged after it
  }
}

template <int GN, bool REVERSE>
hipError_t launch_sweep_g(const SweepArgs& a, int32_t grid, int32_t block, size_t lds,
                          hipStream_t s) {
  if ((block != 256 && block != 512 && block != 1024) || block > kSweepMaxBlock(GN))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep<GN, REVERSE, kStageCh>), dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

template <bool REVERSE>
hipError_t launch_sweep_t(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                          size_t lds, hipStream_t s) {
  switch (gn) {
    case 1: return launch_sweep_g<1, REVERSE>(a, grid, block, lds, s);
    case 2: return launch_sweep_g<2, REVERSE>(a, grid, block, lds, s);
    case 3: return launch_sweep_g<3, REVERSE>(a, grid, block, lds, s);
    case 4: return launch_sweep_g<4, REVERSE>(a, grid, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

// Exponential cell law: with the optical depth tau = kappa V / Aperp (capped at
// 40 for the transmission), the entering power T of a task becomes the exit
// flux density x = T / den, den = Aperp e^{min(tau, 40)}, and the cell average
// is r x, r = Aperp (e^{min(tau, 40)} - 1) / (kappa V) (1 at kappa = 0).
constexpr double kTauCap = 40.0;

__device__ __forceinline__ double exp_den(double ap, double kV) {
  return ap * exp(fmin(kV / ap, kTauCap));
}

__device__ __forceinline__ double exp_r(double ap, double kV) {
  return kV > 0.0 ? ap * expm1(fmin(kV / ap, kTauCap)) / kV : 1.0;
}

// h'(t) for h(t) = (e^t - 1) / t: below 0.5 the power series
// sum_{k>=1} k t^{k-1} / (k+1)! to 18 terms (remainder below 1e-18, Horner
// with the coefficients folded at compile time), above it
// ((t - 1)(e^t - 1) + t) / t^2.
struct DhSeries {
  double c[18];
};

constexpr DhSeries dh_series() {
  DhSeries r{};
  double f = 2.0;  // (k+1)!
  for (int k = 1; k <= 18; ++k) {
    r.c[k - 1] = (double)k / f;
    f *= (double)(k + 2);
  }
  return r;
}

__device__ __forceinline__ double dh_dt(double t) {
  if (t < 0.5) {
    constexpr DhSeries S = dh_series();
    double s = S.c[17];
#pragma unroll
    for (int k = 16; k >= 0; --k) s = s * t + S.c[k];
    return s;
  }
  return ((t - 1.0) * expm1(t) + t) / (t * t);
}

// Per-task denominators (Aperp + kappa V, or the exponential law's den) and
// sources, in schedule order (what the sweep streams).  The sources do not
// depend on the direction: a first pass over the cells packs each cell's
// (kappa, source) per group into one record, so that the pass over the tasks
// reads its Aperp (schedule order) and writes its outputs coalesced, and
// gathers one record and the cell's volume from arrays every direction shares
// (which stay cache resident).  The adjoint source of the exponential law is
// r g, g being the derivative with respect to the cell average.
__global__ __launch_bounds__(256) void k_prep_cells(PrepArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.C_total * a.G) return;
  const int64_t ci = i / a.G;
  const double kap = (double)a.kappa[i];
  double s;
  if (a.emission != nullptr) {
    s = (double)a.emission[i];
    if (a.jsum_prev != nullptr) s += (double)a.albedo * kap * (double)a.vol[ci] * (double)a.jsum_prev[i];
    s *= (double)a.inv_D;
  } else {
    s = (double)a.gsrc[i];
  }
  // invalid inputs raise the DAG's error flag (reported by the next call that
  // synchronises); the kernels run on regardless
  int32_t bad = 0;
  if (!(kap >= 0.0 && kap <= DBL_MAX)) bad |= kErrKappa;
  if (a.emission != nullptr && !((double)a.emission[i] >= 0.0 && (double)a.emission[i] <= DBL_MAX))
    bad |= kErrEmission;
  if (bad != 0) atomicOr(a.flag, bad);
  a.crec[i] = make_float2(a.kappa[i], (float)s);
}

__device__ __forceinline__ int unit_of_block(const int32_t* blk_base, int n_units, int b) {
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk_base[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tasks of a workgroup whose G values per task are staged in LDS, so that the
// workgroup's [tasks][G] block of denominators and sources is written with
// consecutive threads on consecutive words (G up to kPrepStageG; larger G is
// written per task).
constexpr int kPrepStageG = 8;

template <bool EXP_LAW>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  __shared__ float sden[256 * kPrepStageG], ssrc[256 * kPrepStageG];
  const int u = unit_of_block(a.blk_base, a.n_units, blockIdx.x);
  const Unit U = a.units[u];
  const int k0 = (blockIdx.x - a.blk_base[u]) * 256;
  const int k = k0 + threadIdx.x;
  const int G = a.G;
  const bool stage = G <= kPrepStageG;
  int32_t bad = 0;
  if (k < U.n_cells) {
    const int64_t t = U.task_base + k;  // schedule position
    const int64_t ci = (int64_t)U.cell_off + a.sched[t];
    const double V = (double)a.vol_s[t];
    const double ap = (double)a.aperp_s[t];
    // denominator and source of one group from the cell's (kappa, source) record
    auto task = [&](float2 r, float& den_out, float& src_out) {
      const double kap = (double)r.x;
      const double den = EXP_LAW ? exp_den(ap, kap * V) : ap + kap * V;
      double s = (double)r.y;
      if (EXP_LAW && a.emission == nullptr) s *= exp_r(ap, kap * V);
      if (!(den > 0.0 && den <= DBL_MAX)) bad |= kErrCell;
      den_out = (float)den;
      src_out = (float)s;
    };
    if (G == 1) {
      task(a.crec[ci], sden[threadIdx.x], ssrc[threadIdx.x]);
    } else if (stage) {
      // every group's record is loaded before the first is used: unconditional
      // loads (groups past G reread the last one), and the staged results go to
      // LDS, so no store orders them
      float2 r[kPrepStageG];
#pragma unroll
      for (int g = 0; g < kPrepStageG; ++g) r[g] = a.crec[ci * G + min(g, G - 1)];
#pragma unroll
      for (int g = 0; g < kPrepStageG; ++g)
        if (g < G) task(r[g], sden[threadIdx.x * G + g], ssrc[threadIdx.x * G + g]);
    } else {
      for (int g = 0; g < G; ++g) task(a.crec[ci * G + g], a.tden[t * G + g], a.tsrc[t * G + g]);
    }
  }
  if (stage) {
    __syncthreads();
    const int n = min(256, U.n_cells - k0) * G;
    const int64_t base = (U.task_base + k0) * G;
    for (int i = threadIdx.x; i < n; i += 256) {
      a.tden[base + i] = sden[i];
      a.tsrc[base + i] = ssrc[i];
    }
  }
  if (bad != 0) atomicOr(a.flag, bad);
}

// Periodic coupling folded into the sources (PinArgs): one thread per
// (direction, periodic cell, group).
__global__ __launch_bounds__(256) void k_pin(PinArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)a.D * a.n_pc * a.G) return;
  const int g = (int)(i % a.G);
  const int64_t dp = i / a.G;
  const int pc = (int)(dp % a.n_pc);
  const int d = (int)(dp / a.n_pc);
  const int f0 = a.pf_ptr[pc], f1 = a.pf_ptr[pc + 1];
  const float* w = a.pw + (int64_t)d * a.n_pf;
  const float* o = a.other + (int64_t)d * a.C_total * a.G + g;
  float s = 0.0f;
  for (int f = f0; f < f1; ++f) {
    const float wf = w[f];
    if (wf != 0.0f) s = __builtin_fmaf(wf, o[(int64_t)a.pnb[f] * a.G], s);
  }
  const int64_t t = a.ptask[dp];
  float base;
  if (a.capture) {
    base = a.tsrc[t * a.G + g];
    a.pbase[i] = base;
  } else {
    base = a.pbase[i];
  }
  a.tsrc[t * a.G + g] = base + s;
  if (a.pval != nullptr) a.pval[i] = s;
}

// The folded inflow of every (periodic cell, group) summed over directions in
// order, in FP64.
__global__ __launch_bounds__(256) void k_psum(PinArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)a.n_pc * a.G;
  if (i >= n) return;
  double pn = 0.0;
  for (int d = 0; d < a.D; ++d) pn += (double)a.pval[(int64_t)d * n + i];
  a.psum[i] = pn;
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
    const double V = (double)a.vol[c];
    const double kap = (double)a.kappa[cg];
    const bool exp_law = a.law == SWEEP_LAW_EXP;
    double js = 0.0, esc = 0.0, pout = 0.0;
    for (int d = 0; d < a.D; ++d) {
      // phi holds the exit flux density x (phi itself under the upwind law)
      const double ph = (double)a.phi[d * stride + cg];
      const int64_t t = a.units[m * a.D + d].task_base + lc;
      const float2 b = a.bnd[t];
      esc += (double)b.x * ph;
      pout += (double)b.y * ph;
      js += exp_law ? ph * exp_r((double)a.aperp[t], kap * V) : ph;
    }
    // the periodic inflow of the pass (and of the pass before), summed over
    // directions when the pass's sources were folded
    const int pc = a.pc_map != nullptr ? a.pc_map[c] : -1;
    const double pn = pc >= 0 && a.psum != nullptr ? a.psum[(int64_t)pc * G + g] : 0.0;
    {
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
      if (a.with_e) {
        const double po = pc >= 0 && a.psum_prev != nullptr ? a.psum_prev[(int64_t)pc * G + g] : 0.0;
        const double den = pn + po;
        v[6] = den > 0.0 ? fabs(pn - po) / den : 0.0;
        v[7] = fabs(pn - po);
        v[8] = den;
      }
    }
  }
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

// One workgroup per (mesh, group): strided partial sums then a fixed-order
// tree, so the FP64 totals are reproducible.
__global__ __launch_bounds__(256) void k_totals(const double* partial, const int32_t* mesh_blk_base,
                                                int32_t n_meshes, int32_t G, double* totals) {
  __shared__ double sh[256][kNPart];
  const int t = blockIdx.x;
  const int m = t / G, g = t % G;
  double s[kNPart];
  for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
  for (int b = mesh_blk_base[m] + threadIdx.x; b < mesh_blk_base[m + 1]; b += 256)
    for (int k = 0; k < kNPart; ++k) {
      const double x = partial[((int64_t)b * G + g) * kNPart + k];
      if (k == 6) s[k] = fmax(s[k], x); else s[k] += x;
    }
  for (int k = 0; k < kNPart; ++k) sh[threadIdx.x][k] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < kNPart; ++k) {
        const double x = sh[threadIdx.x + w][k];
        sh[threadIdx.x][k] = k == 6 ? fmax(sh[threadIdx.x][k], x) : sh[threadIdx.x][k] + x;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = totals + (int64_t)t * 8;
    for (int k = 0; k < 7; ++k) o[k] = sh[0][k];
    o[7] = sh[0][8] > 0.0 ? sh[0][7] / sh[0][8] : 0.0;
  }
}

__global__ void k_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t n,
                           float* gsrc, double* dk, double* de, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double V = (double)vol[i / G];
  const double ga = (double)dA[i];
  if (!(fabs(ga) <= DBL_MAX && fabs((double)dJ[i]) <= DBL_MAX)) atomicOr(flag, kErrGrad);
  const double ka = (1.0 - (double)albedo) * (double)kappa[i];
  gsrc[i] = (float)((double)dJ[i] * (double)kInv4Pi + ga * ka * V);
  dk[i] = ga * (1.0 - (double)albedo) * V * (double)jsum_last[i];
  de[i] = 0.0;
}

__global__ void k_adj_reduce(AdjReduceArgs a, double* dk, double* de) {
  const int64_t n = a.C_total * a.G;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double V = (double)a.vol[i / a.G];
  double ls = 0.0, dks;
  if (a.law == SWEEP_LAW_EXP) {
    // per direction: -lambda x d(den)/dkappa + g x dr/dkappa, with
    // tau < 40: d(den)/dkappa = V e^tau, dr/dkappa = h'(tau) V / Aperp;
    // tau >= 40: d(den)/dkappa = 0, dr/dkappa = -r / kappa
    const int c = (int)(i / a.G);
    int lo = 0, hi = a.n_meshes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.mesh_off[mid] <= c) lo = mid; else hi = mid - 1;
    }
    // tasks of mesh m: [direction][local cell] from D * (first cell of m)
    const int64_t Cm = a.mesh_off[lo + 1] - a.mesh_off[lo];
    const float* apc = a.aperp + (int64_t)a.D * a.mesh_off[lo] + (c - a.mesh_off[lo]);
    const double kap = (double)a.kappa[i];
    const double kV = kap * V;
    const double g = a.use_g ? (double)a.gsrc[i] : 0.0;
    dks = 0.0;
#pragma unroll 4
    for (int d = 0; d < a.D; ++d) {
      const double l = (double)a.lam[d * n + i];
      const double x = (double)a.phi[d * n + i];
      const double ap = (double)apc[d * Cm];
      const double tau = kV / ap;
      double dden, dr;
      if (tau < kTauCap) {
        dden = V * exp(tau);
        dr = dh_dt(tau) * V / ap;
      } else {
        dden = 0.0;
        dr = -(ap * expm1(kTauCap) / kV) / kap;
      }
      ls += l;
      dks += -l * x * dden + g * x * dr;
    }
  } else {
    double lph = 0.0;
    // (unrolled: the loads of eight directions in flight before the first is used)
#pragma unroll 8
    for (int d = 0; d < a.D; ++d) {
      const double l = (double)a.lam[d * n + i];
      ls += l;
      lph += l * (double)a.phi[d * n + i];
    }
    dks = -V * lph;
  }
  const double prev = a.jsum_prev != nullptr ? (double)a.jsum_prev[i] : 0.0;
  const double alb = (double)a.albedo;
  const double invD = (double)a.inv_D;
  dk[i] += dks + alb * V * ls * prev * invD;
  de[i] += ls * invD;
  const double gn = alb * (double)a.kappa[i] * V * ls * invD;
  a.gsrc_next[i] = (float)(a.accumulate ? (double)a.gsrc_next[i] + gn : gn);
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

LdsLayout sweep_lds_layout(int32_t gn, int32_t ring, int32_t block) {
  LdsLayout L;
  const size_t se = (size_t)kStageCh * block;
  size_t off = (size_t)gn * (ring + 2 + 2 * se) * sizeof(float);  // ring, zero, sink, prefetched
  off = (off + 15) & ~(size_t)15;
  L.stage_off = (int32_t)off;
  off += 2 * (se + 8) * sizeof(int2);  // two staging buffers, 8 entries of padding
  L.bytes = off;
  return L;
}

hipError_t launch_sweep_fwd(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            size_t lds, hipStream_t s) {
  return launch_sweep_t<false>(a, gn, grid, block, lds, s);
}

hipError_t launch_sweep_adj(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            size_t lds, hipStream_t s) {
  return launch_sweep_t<true>(a, gn, grid, block, lds, s);
}

hipError_t launch_prep(const PrepArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_cells, dim3(grid1d(a.C_total * a.G, 256)), dim3(256), 0, s, a);
  if (a.law == SWEEP_LAW_EXP) hipLaunchKernelGGL(k_prep<true>, dim3(n_blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_prep<false>, dim3(n_blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int GN, bool REVERSE>
hipError_t set_lds_g(int32_t bytes) {
  return hipFuncSetAttribute((const void*)k_sweep<GN, REVERSE, kStageCh>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int GN>
hipError_t set_lds_gn(int32_t bytes) {
  hipError_t e;
  if ((e = set_lds_g<GN, false>(bytes)) != hipSuccess) return e;
  return set_lds_g<GN, true>(bytes);
}

hipError_t set_sweep_lds_limit(int32_t bytes) {
  hipError_t e;
  if ((e = set_lds_gn<1>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_gn<2>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_gn<3>(bytes)) != hipSuccess) return e;
  return set_lds_gn<4>(bytes);
}

hipError_t launch_pin(const PinArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.n_pc * a.G;
  if (n <= 0) return hipSuccess;
  if (a.psum != nullptr && a.pval == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pin, dim3(grid1d(n * a.D, 256)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.psum == nullptr) return e;
  hipLaunchKernelGGL(k_psum, dim3(grid1d(n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(n_blocks), dim3(kRedBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_totals(const double* partial, const int32_t* mesh_blk_base, int32_t n_meshes,
                         int32_t G, double* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_totals, dim3(n_meshes * G), dim3(256), 0, s, partial, mesh_blk_base,
                     n_meshes, G, totals);
  return hipGetLastError();
}

hipError_t launch_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t C,
                           float* gsrc, double* dk, double* de, int32_t* flag, hipStream_t s) {
  const int64_t n = C * G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_init, dim3(grid1d(n, 256)), dim3(256), 0, s, dJ, dA, kappa, vol,
                     jsum_last, albedo, G, n, gsrc, dk, de, flag);
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
