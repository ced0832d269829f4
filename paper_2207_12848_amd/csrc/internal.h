// Internal structures shared by the host orchestration and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sweep {

// Bits of the device error flag a DAG keeps: invalid inputs seen by the kernels
// of an asynchronous call, reported by the next call that synchronises.
constexpr int32_t kErrKappa = 1;     // kappa negative or not finite
constexpr int32_t kErrEmission = 2;  // emission negative or not finite
constexpr int32_t kErrCell = 4;      // a task's denominator (Aperp + kappa V) not positive and finite
constexpr int32_t kErrGrad = 8;      // dL/dJ or dL/dabsorbed not finite

// Largest byte size of any array the sweep kernels address through a buffer
// resource (32-bit offsets; offsets from kOob up stay past the end).
constexpr int64_t kMaxBufBytes = 0x7fffffe0;

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
  const int32_t* face_twin;  // matching half-face of the neighbour (scheme (b) only)
  const int32_t* fcode;  // per face: neighbour code (see k_face_codes)
  int64_t face_off;      // first face of the mesh in the concatenated per-face arrays
  int64_t n_faces;
  int32_t n_cells;
  int32_t cell_off;
};

struct DagBuildArgs {
  const Unit* units;
  int32_t n_units;
  int32_t D;
  const MeshDev* meshes;
  const double* dirs;  // [D][3]
  double eps;
  int32_t scheme;      // SWEEP_SCHEME_AREA (a) or SWEEP_SCHEME_ALIGNED (b)
  int32_t n_aligned;   // scheme (b): outflow faces that share a cell's outflow (1..kMaxAligned)
  const int32_t* blk_base;  // [n_units+1] first block of each unit (cell-range kernels)
  const int32_t* cblk_mesh;  // cell-order kernels: mesh and first cell of every block
  const int32_t* cblk_c0;
  int32_t dn_width;          // width of the fixed-width downwind rows (16 or 32)
  int32_t dn_chunks;         // chunks of 4 row entries that may hold a downwind cell
  int32_t* dn_ovf;           // overflow lists of full rows: [count, cells...]
  int32_t* dn_ovf_top;       // next free int of dn_ovf (atomic)
  int64_t dn_ovf_cap;        // ints of dn_ovf for lists (more: the pool has run out)
  int64_t* big;              // tasks with 15 or more upwind dependencies
  int32_t* big_top;          // their number (atomic)
  int32_t max_faces;         // most half-faces of any cell
  int32_t* dnw;              // [T][dn_width] downwind cells of every task (-1 padded)
  int64_t dn_sentinel;       // offset in dnw of a row of -1 (4 * kRowChunks entries)
  int32_t* stats;            // [0] max in-degree, [1] max out-degree (atomic max)
  unsigned long long* ent_tot;  // [0] upwind-row entries, [1] downwind-row entries (all tasks)
  // per task, cell order within the unit (the upwind row's length is indeg)
  int32_t* indeg;
  int32_t* rowlen_dn;
  float* aperp;
  float* aperp_s;  // the same per task in schedule order (written by k_gather_len)
  float* vol_s;    // the cell's volume per task, schedule order (written by k_gather_len)
  // per (direction, face) of every mesh, at D * face_off + d * n_faces + f: the face
  // weight w = A |Omega . n| rounded once to FP32 from FP64, with the face's class
  // in its sign: outflow +w, inflow -w, neither NaN
  float* wface;
  float2* bnd;  // (sum of w over wall outflow faces, over periodic outflow faces)
  int32_t* cnt;    // [T] words: Kahn's counters kept in global memory
  int32_t* inv;    // cell -> position in the unit's schedule (written by k_sort_levels)
  // per task, schedule order within the unit
  int32_t* sched;  // position -> cell
  int32_t* lp;     // level pointers
  int32_t* depth;  // [n_units]
  int32_t* err;    // set to 1 if a unit could not be fully ordered
  int64_t* lev_up;  // per unit level table: first upwind-row entry of each level
  int64_t* lev_dn;
  // periodic half-faces (the lists that fold the coupling between periodic passes
  // into the sources, built after the rows; see PinArgs)
  int32_t* npf;      // [C_total + 1] periodic half-faces of every cell (scan input)
  int32_t* pflag;    // [C_total + 1] 1 for a cell with periodic half-faces (scan input)
  const int64_t* pf_off;  // [C_total + 1] exclusive scan of npf
  const int64_t* pc_off;  // [C_total + 1] exclusive scan of pflag
  int32_t n_pc;      // periodic cells
  int64_t n_pf;      // periodic half-faces
  int32_t* pcell;    // [n_pc] global cell id
  int32_t* pf_ptr;   // [n_pc + 1] first half-face of each periodic cell
  int32_t* pface;    // [n_pf] the half-face (index within its mesh; build only)
  int32_t* pnb;      // [n_pf] partner cell across the half-face (global id)
  float* pwf;        // [D][n_pf] inflow weight (0 where the half-face is no inflow)
  float* pwa;        // [D][n_pf] outflow weight (0 where the half-face is no outflow)
  int32_t* ptask;    // [D][n_pc] task of (direction, periodic cell)
  int32_t* pc_map;   // [C_total] periodic cell index of every cell, -1 for the others
  int32_t* len_up;  // [T+1] row lengths in schedule order (scan input)
  int32_t* len_dn;  // [T+1]
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
  // groups [g0, g0 + n_chunks x GN) are swept as n_chunks independent chunks of
  // GN packed groups: work item i is unit unit_order[i / n_chunks], groups from
  // g0 + (i % n_chunks) GN (the chunks of the longest units first)
  int32_t n_chunks;
  int32_t* work_counter;  // persistent form: next work item; nullptr: item = blockIdx.x
  const int32_t* sched;
  // steps of the level-synchronous sweep (see k_steps): unit u's steps start at
  // step_base[u]; step i covers schedule positions [step_k[i], step_k[i + 1]) and
  // row entries [step_e[i], step_e[i + 1]) (upwind rows forward, downwind adjoint)
  const int32_t* step_k;
  const int64_t* step_e;
  const int64_t* step_base;
  const int32_t* n_steps;
  const int64_t* row_ptr;  // up_ptr (forward) or dn_ptr (adjoint)
  const int2* ent;         // up (forward) or dn (adjoint)
  int64_t n_ent;           // entries in `ent`
  const float* tden;       // [T][G] schedule order: Aperp + kappa V
  const float* tsrc;       // [T][G] schedule order: source of the task (periodic
                           // coupling included, see PinArgs)
  float* out;              // phi (forward) or lambda (adjoint), [D][C][G]
  float* out_s;            // the same values in schedule order, [T][G]
  int64_t C_total;
  int32_t G;       // group stride
  int32_t g0;      // first group handled by this launch (see n_chunks)
  int32_t D;
  int32_t ring_mask;
  int32_t stage_off;      // byte offset of the staging buffers in the dynamic LDS
};

// Per-call preparation of the per-task denominators and sources, written in
// schedule order.
struct PrepArgs {
  const Unit* units;
  int32_t n_units;
  const int32_t* blk_base;
  const int32_t* sched;
  const float* aperp_s;    // per task, schedule order
  const float* vol_s;      // the cell's volume per task, schedule order
  const float* kappa;      // [C][G]
  const float* vol;        // [C]
  const float* emission;   // forward source [C][G] (divided by D), or
  const float* gsrc;       // adjoint source [C][G] (used when emission == nullptr)
  const float* jsum_prev;  // [C][G] or nullptr
  float albedo;
  float inv_D;
  int32_t G;
  int32_t law;             // SWEEP_LAW_UPWIND / SWEEP_LAW_EXP
  int64_t C_total;
  int32_t* flag;           // device error bits (atomicOr): kErrKappa, kErrEmission, kErrCell
  float2* crec;            // [C_total][G] scratch: (kappa, source of the cell)
  float* tden;             // [T][G] schedule order
  float* tsrc;             // [T][G] schedule order
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
  const int32_t* pc_map;     // [C_total] periodic cell index or -1 (nullptr: no periodic inflow)
  const double* psum;        // [n_pc][G] periodic inflow of the pass summed over directions
  const double* psum_prev;   // [n_pc][G] the same of the pass before, or nullptr (zero inflow)
  int32_t with_e;            // 1: E of the pass against the pass before (sec. 2.7)
  const float2* bnd;         // per task, cell order
  const float* aperp;        // per task, cell order
  int32_t law;
  const float* kappa;
  const float* emission;
  const float* vol;
  const float* jsum_prev;    // [C][G] or nullptr
  float albedo;
  float* jsum;               // [C][G] out
  float* J;                  // out
  float* absorbed;           // out
  double* partial;           // [n_blocks][G][9]
  int32_t cells_per_block;
};

// Periodic coupling of a pass, folded into its sources: a task of a periodic
// cell takes, through each periodic half-face that carries radiation into it
// (forward) or out of it (adjoint), w times the other pass's value at the
// partner cell (forward: the previous pass's exit value; adjoint: the later
// pass's lambda).  These values are final before the pass starts, so the sum
// (an FP32 FMA chain in face order) is added to the task's source beforehand
// and the sweep itself reads no other pass.
struct PinArgs {
  int32_t D;
  int32_t G;
  int64_t C_total;
  int32_t n_pc;
  int64_t n_pf;
  const int32_t* pf_ptr;   // [n_pc + 1]
  const int32_t* pnb;      // [n_pf]
  const float* pw;         // [D][n_pf] the pass's weights (inflow or outflow)
  const int32_t* ptask;    // [D][n_pc]
  const float* other;      // [D][C_total][G] the other pass's values
  float* tsrc;             // [T][G] sources of the pass
  float* pbase;            // [D][n_pc][G] the periodic tasks' own sources
  int32_t capture;         // 1: tsrc holds the own sources (save them), 0: take pbase
  float* pval;             // [D][n_pc][G] the folded sums (needed with psum)
  double* psum;            // [n_pc][G] out: their sum over directions (FP64), or nullptr
};

struct AdjReduceArgs {
  int32_t D;
  int32_t G;
  int64_t C_total;
  int32_t law;
  int32_t n_meshes;
  const int32_t* mesh_off; // [n_meshes + 1] first global cell of each mesh
  const float* aperp;      // per task: unit (m, d) starts at D * mesh_off[m] + d * cells(m)
  const float* gsrc;       // [C][G] adjoint source of this iteration (dL/d cell average)
  int32_t use_g;           // this pass carries the loss (its g enters the kappa derivative)
  int32_t accumulate;      // add to gsrc_next (earlier periodic passes) instead of writing it
  const float* lam;        // [D][C][G]
  const float* phi;        // [D][C][G]
  const float* kappa;
  const float* vol;
  const float* jsum_prev;  // [C][G] sum_d phi^{i-1} or nullptr
  float albedo;
  float inv_D;
  float* gsrc_next;        // adjoint source of the previous iteration
};

// Photoionisation chemistry step (chem.hip).
struct IonArgs {
  int64_t n;               // cells
  const float* vol;        // [n] mesh units
  const float* absorbed;   // [n] photons/s in units of photon_rate
  double* neutral;         // [n] neutral fraction y
  float* kappa;            // [n] out: n_H y sigma_H length_unit
  double n_H, sigma_H, alpha_B, photon_rate, length_unit;
  double l3;               // length_unit^3
};

// launchers (kernels in dag.hip / sweep.hip / chem.hip)
hipError_t launch_ion_limit(const IonArgs& a, unsigned long long* out, hipStream_t s);
// Device address of the current device's scratch word of sweep_ion_step_noalloc
// (looked up once per device).
hipError_t ion_scratch(unsigned long long** out);
hipError_t launch_ion_update(const IonArgs& a, double dt, hipStream_t s);
constexpr int kTileCellsHost = 32;  // cells per tile of the cell-order build kernels
hipError_t launch_count(const DagBuildArgs& a, int32_t n_cblocks, int32_t lds_limit, hipStream_t s);
constexpr int kMaxAligned = 4;  // most faces scheme (b) may share the outflow over
hipError_t launch_kahn(const DagBuildArgs& a, bool lds_counters, int32_t max_cells, hipStream_t s);
hipError_t launch_fill(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s);
// out[0] = max faces of a cell, out[1] += overflow ints for rows of row_cap entries
hipError_t launch_face_stats(const int64_t* face_ptr, int32_t n_cells, int32_t row_cap, int32_t n_dirs,
                             unsigned long long* out, hipStream_t s);
hipError_t launch_face_codes(const MeshDev& m, int32_t* fcode, hipStream_t s);
// Sorts every level of the schedule by cell id and writes the inverse schedule.
hipError_t launch_sort_levels(const DagBuildArgs& a, hipStream_t s);
hipError_t launch_gather_len(const DagBuildArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_mark(const DagBuildArgs& a, int32_t n_big, hipStream_t s);
size_t count_lds_bytes(int max_faces, int dn_width);
hipError_t launch_level_entries(const DagBuildArgs& a, hipStream_t s);
// out[2u], out[2u + 1]: upwind and downwind row entries of unit u
hipError_t launch_unit_entries(const Unit* units, int32_t n_units, const int64_t* up_ptr,
                               const int64_t* dn_ptr, int64_t* out, hipStream_t s);
// width[l] += tasks at level l of every unit of `mesh` (all meshes if mesh < 0), l < n_levels
hipError_t launch_level_widths(const Unit* units, int32_t n_units, const int32_t* lp, int32_t mesh,
                               int64_t* width, int32_t n_levels, hipStream_t s);
hipError_t launch_ion_kappa(const IonArgs& a, hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_scan_len(const int32_t* in, int64_t* out, int64_t n, void* tmp, size_t* tmp_bytes,
                           hipStream_t s);
hipError_t launch_d2f(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);

hipError_t launch_sweep_fwd(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            size_t lds_bytes, hipStream_t s);
hipError_t launch_sweep_adj(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            size_t lds_bytes, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, int32_t n_blocks, hipStream_t s);
hipError_t launch_pin(const PinArgs& a, hipStream_t s);
hipError_t launch_pcount(const DagBuildArgs& a, const MeshDev& m, hipStream_t s);
hipError_t launch_plist(const DagBuildArgs& a, const MeshDev& m, hipStream_t s);
hipError_t launch_pdir(const DagBuildArgs& a, const MeshDev& m, int32_t mesh, hipStream_t s);
hipError_t launch_totals(const double* partial, const int32_t* mesh_blk_base, int32_t n_meshes,
                         int32_t G, double* totals, hipStream_t s);
hipError_t launch_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t C,
                           float* gsrc, double* dk, double* de, int32_t* flag, hipStream_t s);
hipError_t launch_adj_reduce(const AdjReduceArgs& a, double* dk, double* de, hipStream_t s);
hipError_t launch_d2f_pair(const double* a, const double* b, float* oa, float* ob, int64_t n,
                           hipStream_t s);
hipError_t set_sweep_lds_limit(int32_t bytes);
// Row entries each sweep thread stages per step (a step holds at most
// kStageCh x threads - 8 entries in LDS).  Twice as many (fewer, larger steps,
// which the LDS holds with two packed groups) measured slower on the clustered
// 2M-cell mesh: each step then keeps more loads in flight than the memory
// system returns in time.
constexpr int kStageCh = 4;
// Largest sweep workgroup for gn packed groups: one group fits 1024 threads'
// registers (128 VGPRs each), more groups need the 256 VGPRs of 512 threads.
constexpr int kSweepMaxBlock(int gn) { return gn == 1 ? 1024 : 512; }
// Dynamic LDS layout of a sweep workgroup of `block` threads: values (ring
// slots, a zero slot, a sink, 2 x kStageCh x block prefetched slots) x gn FP32,
// then two staging buffers of kStageCh x block + 8 entries.
struct LdsLayout {
  int32_t stage_off;
  size_t bytes;
};
LdsLayout sweep_lds_layout(int32_t gn, int32_t ring, int32_t block);
// Steps of the level-synchronous sweep with at most cap_t tasks and about
// cap_e row entries each (see k_steps), written from step_base[u] per unit.
hipError_t launch_steps(const Unit* units, int32_t n_units, const int32_t* lp, const int64_t* lev_up,
                        const int64_t* lev_dn, const int64_t* up_ptr, const int64_t* dn_ptr,
                        const int64_t* step_base, int32_t cap_t, int32_t cap_e, int32_t* step_k,
                        int64_t* step_eu, int64_t* step_ed, int32_t* n_steps, hipStream_t s);

}  // namespace sweep
