// Internal descriptors shared by the host library and the gfx950 kernels.
// All device arrays are structure-of-arrays: a [k][n] array stores component c
// of item i at c*n + i, so that consecutive threads read consecutive words.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

// In the kernels' device code the device pointers held by these descriptors
// are global-address-space pointers, so that their loads and stores are
// global (not flat) memory instructions: a wait for LDS results then does not
// also wait for outstanding global loads.
#if defined(__HIP_DEVICE_COMPILE__) && defined(T2R_KERNEL_TU)
#define T2R_G __attribute__((address_space(1)))
#else
#define T2R_G
#endif

namespace t2r {

// Tet tiles: a workgroup stages one tile's vertices in LDS, evaluates its tets
// and accumulates per-vertex sums with LDS atomics before one global flush.
constexpr int kTileTets = 1024;
constexpr int kTileVerts = 512;   // local vertex ids are 16-bit
constexpr int kMaxBlock = 1024;

// Workgroups take envs in order of decreasing expected cost (indenter motion of
// the launch, scaled by the env's previous cost per unit motion), so the
// longest solves start first and the launch ends with short ones.
// Up to kOrderMax envs are sorted (one workgroup); beyond that envs go in id order.
constexpr int kOrderMax = 8192;

// Contact slots: the gel and indenter vertices touched by an env's coarse pair
// list get dense ids (below kGelSlots and kIndSlots), so pair passes stage
// their positions in LDS (in the tile's storage), accumulate gradients there
// and write each gel vertex once per pass. A pair record packs the slot of each
// of its four points (kRecBits each) and its kind; a friction record packs
// 10-bit gel and indenter slots, kNoSlot10 marking an unused point.
constexpr int kGelSlots = 512;
constexpr int kIndSlots = 1024;
constexpr int kRecBits = 11;
constexpr uint32_t kNoSlot10 = 1023;

// Pair kinds of the contact list (top three bits of the first word).
constexpr int kVF = 0;   // gel surface vertex  vs indenter triangle
constexpr int kFV = 1;   // indenter vertex     vs gel surface triangle
constexpr int kEE = 2;   // gel surface edge    vs indenter edge
constexpr int kGVF = 3;  // gel surface vertex  vs gel surface triangle (self-contact)
constexpr int kGEE = 4;  // gel surface edge    vs gel surface edge (self-contact)
constexpr int kKindShift = 29;
constexpr int kPrimMask = (1 << kKindShift) - 1;

// Tile vertex flags.
constexpr uint8_t kFirstTouch = 1;  // this tile writes the vertex first (store, not add)
constexpr uint8_t kLastTouch = 2;   // this tile writes it last
constexpr uint8_t kFixedLast = 4;   // last touch of a fixed vertex: gradient 0, diagonal 1

struct Grid {              // uniform grid over an indenter's local bounding box
  double origin[3];
  double inv_cell;         // 1 / cell edge (cells are cubes)
  int dims[3];
  const T2R_G int* start;        // [ncell+1] CSR offsets
  const T2R_G int* items;        // primitive ids per cell
  const T2R_G double* box;       // [6][n_prim]: lo xyz, hi xyz of each primitive (local frame)
  int n_prim;
};

struct GelDev {
  int n_v, n_t, n_tiles, n_sv, n_se, n_sf, n_m;
  double vol_total;        // sum of rest volumes
  double diag_rest_max;    // largest rest elastic diagonal entry for mu = 1, lam = 0
  const T2R_G double* X;         // [3][n_v]
  const T2R_G uint8_t* fixed;    // [n_v]
  const T2R_G int* tet;          // [4][n_t] global vertex ids, tiled order
  const T2R_G uint64_t* tet_local;  // [n_t] four 16-bit local ids
  const T2R_G double* Dinv;      // [9][n_t] Dm^-1 row-major entries
  const T2R_G double* vol;       // [n_t]
  const T2R_G float* Dinv32;     // [9][n_t] FP32 copy (mixed precision)
  const T2R_G float* vol32;      // [n_t]
  const T2R_G int* tile_tet;     // [n_tiles+1]
  const T2R_G int* tile_vstart;  // [n_tiles+1]
  const T2R_G int* tile_verts;   // global vertex ids of each tile
  const T2R_G uint8_t* tile_flags;  // kFirstTouch | kLastTouch | kFixedLast per tile vertex
  const T2R_G int* surf_v;       // [n_sv]
  const T2R_G int* surf_e;       // [2][n_se]
  const T2R_G int* surf_f;       // [3][n_sf]
  const T2R_G int* marker_tri;   // [3][n_m]
  const T2R_G double* marker_w;  // [3][n_m]
  const T2R_G double* vmass;     // [n_v] sum of V_e / 4 over the vertex's tets (lumped mass / density)
};

struct IndDev {
  int n_v, n_f, n_e;
  double r_max;            // largest |y| over local vertices
  double box_lo[3], box_hi[3];  // local bounding box
  const T2R_G double* Y;         // [3][n_v]
  const T2R_G int* tri;          // [3][n_f]
  const T2R_G int* edge;         // [2][n_e]
  Grid gv, ge, gf;         // grids of vertices, edges and triangles
};

struct EnvDev {
  int gel, ind;
  double mu, lam, mu_f, eps_v, dhat, kappa;
  long long voff;          // offset (doubles) of this env's [3][n_v] block in each state array
  long long poff;          // offset of its pair list
  long long foff;          // offset of its friction list
  long long moff;          // offset (markers) in the marker output
  long long ooff;          // offset of its outer (coarse) candidate list
  long long snoff;         // offset of its two surface-vertex snapshots (6 n_sv doubles)
  long long vtxoff;        // vertex offset (voff / 3) of its vertex map
  long long imoff;         // offset of its indenter vertex map
  int pair_cap, fric_cap, outer_cap;
  int has_off;             // a rigid pose offset is set (t2r_set_pose_offsets)
  double off[6];           // its translation dt (mm) and rotation vector dw (rad)
  double density;          // mass density of the dynamic form (t/mm^3); 0: the option's
};

struct FricPair {          // lagged friction data of one pair (Supp. A, eq. friction_energy)
  int gv[3];               // gel vertex ids (-1 unused)
  int iv[3];               // indenter vertex ids (-1 unused)
  double a[3];             // gel-side closest-point weights
  double c[3];             // indenter-side closest-point weights
  double n[3];             // unit normal, indenter closest point -> gel closest point
  double base[3];          // sum a x_prev - sum c y(q_prev)
  double mulam;            // mu_f * lambda = -mu_f kappa b'(d) at the lag
  uint64_t slot;           // gel slots of gv[0..2] (bits 0-29), indenter slots of iv[0..2] (bits 32-61)
};

struct ListState {         // neighbour lists kept across load steps
  double pose_o[7];        // indenter pose when the outer list was built
  double pose_i[7];        // ... and when the inner list was built
  int n_outer, n_inner, valid_o, valid_i;
  int n_slots, n_islots;   // gel and indenter contact slots of the outer list
  int slots_ok;            // 0: too many vertices; pair passes gather from global memory
};

struct EnvStats {
  int status, iters, substeps, restarts, halvings, reculls, n_candidates, n_active,
      n_friction, max_solve_iters, outer_builds, n_outer;
  double d_min, residual, energy;
  double phase_ms[10];     // see t2r_env_stats
  double list_fill;        // largest list length / capacity seen in the launch
  int evals, reserved;     // evaluation passes (energy + curvature) of the launch
};

struct StepParams {
  const T2R_G GelDev* gels;
  const T2R_G IndDev* inds;
  const T2R_G EnvDev* envs;
  int n_env;
  // state
  T2R_G double* x;               // [sum 3 n_v]
  T2R_G double* xprev;
  T2R_G double* g0;
  T2R_G double* g1;
  T2R_G double* diag;
  T2R_G double* p;
  T2R_G double* pose_prev;       // [n_env][7]
  T2R_G double* pose_lag;        // [n_env][7] q_{s-1} of the last load step (friction lag pose)
  T2R_G double* adj;             // [sum 3 n_v] adjoint scratch vector
  T2R_G int2* pairs;             // [sum pair_cap]
  T2R_G double* pair_d;          // [sum pair_cap] distance of each candidate at the current x
  T2R_G int2* outer;             // [sum outer_cap] coarse candidates (wider radius, rebuilt rarely)
  T2R_G ListState* lists;        // [n_env]
  T2R_G double* xsnap;           // [sum 6 n_sv] surface positions when the lists were built
  T2R_G FricPair* fric;          // [sum fric_cap]
  T2R_G int* vmap;               // [sum n_v] gel vertex -> slot + 1 while slots are built, else 0
  T2R_G int* imap;               // [sum indenter n_v] ... for indenter vertices
  T2R_G uint64_t* oslot;         // [sum outer_cap] pair record of each outer pair
  T2R_G uint64_t* pslot;         // [sum pair_cap] ... of each inner pair
  T2R_G int* slot_v;             // [n_env][kGelSlots] gel vertex of each slot
  T2R_G int* islot_v;            // [n_env][kIndSlots] indenter vertex of each slot
  T2R_G EnvStats* stats;         // [n_env]
  const T2R_G int* order;        // [n_env] env of each workgroup (longest expected first) or null
  // inputs / outputs
  const T2R_G double* pose_in;   // [n_steps][n_env][7] (motion_mode 0)
  // motion_mode 1: motion_in [n_env][6] = linear and world-frame angular
  // velocity, applied for motion_dt over the launch's n_steps load steps from
  // each env's pose at the launch start; 2: motion_in and motion_in2 [n_env][7]
  // = poses at the start and end of a motion whose relative displacement
  // (t1 - t0, q1 q0^-1) is applied the same way
  int motion_mode;
  const T2R_G double* motion_in;
  const T2R_G double* motion_in2;
  double motion_dt;
  const T2R_G int* env_mask;     // [n_env] or null
  T2R_G double* markers_out;     // [n_steps][sum n_m][3] or null
  long long markers_stride;      // doubles per load step in markers_out (3 sum n_m)
  int n_steps;                   // load steps in this launch
  T2R_G double* x_out;           // [sum n_v][3] or null
  T2R_G int* status_out;         // [n_steps][n_env] or null
  T2R_G long long* x_out_off;    // [n_env] vertex offsets into x_out
  // options
  double clock_khz;        // wall-clock counter rate (phase timers)
  double tol, substep_tol;
  int max_iters, max_substeps, precision, armijo;
  int ee_moll;                   // weight edge-edge barriers by the parallel-edge mollifier
  double outer_mult;             // coarse list margin beyond dhat, in multiples of dhat
  int det;                       // deterministic summation and list order
  int selfc;                     // barriers between gel surface primitives too
  long long max_evals;           // energy + curvature passes per env per launch (<= 0: no limit)
  int warm_start;                // extrapolate the previous load step's displacement
  T2R_G double* gap0;            // [n_env] d_min at the start of the env's previous load step (0: unknown)
  T2R_G double* vel;             // [sum 3 n_v] velocities of the dynamic form
  double inertia_w;              // density / dt^2 (0: quasi-static)
  double dt;                     // time step of the dynamic form
  // trajectory tape: entry k holds every env's positions ([sum 3 n_v], the
  // layout of x) and pose ([n_env][7]) after the k-th recorded load step
  // (entry 0: the state when recording started)
  T2R_G double* tape_x;          // [entries][sum 3 n_v] or null (step kernel: no recording)
  T2R_G double* tape_q;          // [entries][n_env][7]
  long long tape_stride;         // doubles per positions entry (sum 3 n_v)
  int tape_k0;                   // step kernel: load step k of the launch writes entry tape_k0 + k + 1
  // adjoint
  const T2R_G double* dL_du;     // [bw_steps][sum n_m][3] (markers_stride doubles per step)
  T2R_G double* grad_out;        // [n_env][9]
  double cg_tol;                 // relative residual of the adjoint solve
  int bw_steps;                  // load steps differentiated (the last bw_steps recorded)
  int bw_last;                   // tape entry of the last step's equilibrium
};

struct EvalParams {
  StepParams sp;           // state pointers point at scratch copies
  int env;
  const T2R_G double* pose;      // device [7]
  const T2R_G double* pose_lag;  // device [7]
  int has_lag, has_p;
  T2R_G double* grad_out;        // [n_v][3] or null
  T2R_G double* diag_out;
  T2R_G double* scalars_out;     // [8]
};

}  // namespace t2r

extern "C" {
hipError_t t2r_launch_step(const t2r::StepParams* p, int block, hipStream_t stream);
hipError_t t2r_launch_order(const t2r::StepParams* p, int* order, double* motion, hipStream_t stream);
hipError_t t2r_launch_backward(const t2r::StepParams* p, int block, hipStream_t stream);
hipError_t t2r_launch_eval(const t2r::EvalParams* p, int block, hipStream_t stream);
hipError_t t2r_launch_pack_state(const t2r::StepParams* p, const double* in, double* out,
                                 const long long* state_off, int direction, hipStream_t stream);
hipError_t t2r_launch_aos_to_soa(const double* in, double* out, int nv, hipStream_t stream);
hipError_t t2r_static_scratch(int device, double** ptr, size_t* n_doubles);
size_t t2r_static_scratch_capacity();
}
