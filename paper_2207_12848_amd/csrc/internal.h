// Internal structures shared by the host orchestration and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sweep {

// One (mesh, direction) sweep.  Task arrays of unit u occupy
// [task_base, task_base + n_cells); its level pointers [lp_base, lp_base + depth + 2).
struct Unit {
  int64_t task_base;
  int64_t lp_base;
  int32_t n_cells;
  int32_t depth;
  int32_t dir;
  int32_t mesh;
  int32_t cell_off;  // global id of the mesh's first cell
  int32_t pad;
};

// Device view of one input mesh (valid during the build only).
struct MeshDev {
  const int64_t* face_ptr;
  const int32_t* face_nbr;
  const int8_t* face_shift;  // nullptr: no periodic faces
  const double* face_area;
  const double* face_normal;
  const double* cell_volume;
  int32_t n_cells;
  int32_t cell_off;
};

struct DagBuildArgs {
  const Unit* units;
  int32_t n_units;
  const MeshDev* meshes;
  const double* dirs;  // [D][3]
  double eps;
  const int32_t* blk_base;  // [n_units+1] first block of each unit (cell-range kernels)
  // per task, cell order within the unit
  int32_t* indeg;
  int32_t* rowlen_up;
  int32_t* rowlen_dn;
  float* aperp;
  float2* bnd;  // (sum of w over wall outflow faces, over periodic outflow faces)
  int32_t* cnt;
  int32_t* inv;    // cell -> position in the unit's schedule
  int32_t* level;
  // per task, schedule order within the unit
  int32_t* sched;  // position -> cell
  int32_t* lp;     // level pointers
  int32_t* depth;  // [n_units]
  int32_t* err;    // set to 1 if a unit could not be fully ordered
  int64_t* len_up;  // [T+1] row lengths in schedule order (scan input)
  int64_t* len_dn;  // [T+1]
  int64_t* up_ptr;  // [T+1]
  int64_t* dn_ptr;  // [T+1]
  int2* up;         // (position of the upwind task | -(partner cell + 1) for periodic inflow, w)
  int2* dn;         // (position of the downwind task, w)
};

// Arguments of the forward and adjoint sweep kernels.
struct SweepArgs {
  const Unit* units;
  const int32_t* unit_order;  // processing order of the units (longest first)
  int32_t n_units;
  int32_t* work_counter;  // persistent form: next unit to take; nullptr: unit = blockIdx.x
  const int32_t* sched;
  const int32_t* lp;
  const int64_t* row_ptr;  // up_ptr (forward) or dn_ptr (adjoint)
  const int2* ent;         // up (forward) or dn (adjoint)
  const float* aperp;      // per task, cell order
  const float* kappa;      // [C][G]
  const float* src;        // forward: emission [C][G]; adjoint: adjoint source [C][G]
  const float* vol;        // [C]
  const float* jsum_prev;  // forward: [C][G] sum_d phi of the previous iteration, or nullptr
  const float* phi_prev;   // forward: [D][C][G] previous periodic pass, or nullptr (zero inflow)
  float* out;              // phi (forward) or lambda (adjoint), [D][C][G]
  float* pin;              // forward, periodic: inflow through periodic faces per task, or nullptr
  int64_t C_total;
  int32_t G;       // group stride
  int32_t g0;      // first group handled by this launch
  int32_t D;
  int32_t ring_mask;
  float albedo;
  float inv_D;
};

// Reduction over directions (per cell and group).
struct ReduceArgs {
  const Unit* units;
  int32_t D;
  int32_t G;
  int64_t C_total;
  const int32_t* blk_mesh;   // [n_blocks]
  const int32_t* blk_cell0;  // [n_blocks] global first cell of the block
  const int32_t* mesh_off;   // [n_meshes+1]
  const int32_t* mesh_cells;  // [n_meshes]
  const float* phi;          // [D][C][G]
  const float* pin;          // [D][C][G] or nullptr
  const double* pin_prev;    // [C][G] or nullptr
  const float2* bnd;         // per task, cell order
  const float* kappa;
  const float* emission;
  const float* vol;
  const float* jsum_prev;    // [C][G] or nullptr
  float albedo;
  float* jsum;               // [C][G] out
  float* J;                  // out
  float* absorbed;           // out
  double* pin_sum;           // [C][G] out (periodic pass bookkeeping) or nullptr
  double* partial;           // [n_blocks][G][9]
  int32_t cells_per_block;
  int32_t last;              // 1: final pass (write J/absorbed/totals), 0: only pin_sum
};

struct AdjReduceArgs {
  int32_t D;
  int32_t G;
  int64_t C_total;
  const float* lam;        // [D][C][G]
  const float* phi;        // [D][C][G]
  const float* kappa;
  const float* vol;
  const float* jsum_prev;  // [C][G] sum_d phi^{i-1} or nullptr
  float albedo;
  float inv_D;
  float* gsrc_next;        // adjoint source of the previous iteration
};

// launchers (kernels in dag.hip / sweep.hip)
hipError_t launch_count(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_kahn(const DagBuildArgs& a, hipStream_t s);
hipError_t launch_gather_len(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_fill(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, size_t* tmp_bytes,
                           hipStream_t s);
hipError_t launch_d2f(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);

hipError_t launch_sweep_fwd(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            int32_t ring, hipStream_t s);
hipError_t launch_sweep_adj(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            int32_t ring, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_totals(const double* partial, const int32_t* mesh_blk_base, int32_t n_meshes,
                         int32_t G, double* totals, hipStream_t s);
hipError_t launch_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t C,
                           float* gsrc, double* dk, double* de, hipStream_t s);
hipError_t launch_adj_reduce(const AdjReduceArgs& a, double* dk, double* de, hipStream_t s);
hipError_t launch_d2f_pair(const double* a, const double* b, float* oa, float* ob, int64_t n,
                           hipStream_t s);
hipError_t set_sweep_lds_limit(int32_t bytes);
size_t sweep_lds_bytes(int32_t gn, int32_t ring);

}  // namespace sweep
