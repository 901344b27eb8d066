// gfx950 kernels of the PNCG-IPC gel solver.
//
// One workgroup owns one environment for a whole load step: continuation over
// the indenter motion, broad phase, every PNCG iteration and the marker output
// run in one launch with only workgroup barriers, so the iteration loop stays
// on the device and an env's vectors are touched by a single CU (its L1 and the
// XCD's L2). Thousands of environments fill the 256 CUs.
//
// Per PNCG iteration (Supp. A, eqs. dk_direction, step_size):
//   curvature pass   p^T H p over tets (LDS-staged tiles) and contact pairs
//   CCD pass         conservative step bound over candidate pairs
//   eval pass        Pi, grad, diag(H) at x + alpha p (tiles + pairs + friction),
//                    repeated with alpha/2 until feasible and decreasing
//   dots pass        x += alpha p, P = diag^-1, DK dot products, |P g|_inf
//   direction pass   p = -P g + beta p
#include <float.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include <hip/hip_runtime.h>

#define T2R_KERNEL_TU 1
#include "t2r_internal.h"
#include "t2r_math.h"

namespace t2r {

constexpr double kInf = 1.0e300;
constexpr double kArmijoC = 1e-4;
constexpr double kEnergyGuard = 1e-13;     // x mu * total volume (energies are FP64 in both modes)
constexpr double kDiagFloor = 1e-12;       // x mu * largest rest diagonal (mu = 1 part)
constexpr double kYpMin = 1e-30;
constexpr int kMaxHalvings = 30;
// Entries of a per-vertex vector a thread loads per trip in the streaming passes
// of the direction update.
constexpr int kVecUnroll = 4;
constexpr double kCcdGap = 0.1;            // keep every pair at >= 10% of its gap
constexpr int kCcdMaxAdvance = 64;
constexpr double kSqrt3 = 1.7320508075688772;

// Status bits (mirror T2R_ENV_* in t2r.h).
constexpr int kConverged = 1, kMaxIter = 2, kInfeasible = 4, kNonFinite = 8, kOverflow = 16,
              kLineSearch = 32, kSubsteps = 64, kSkipped = 128, kBudget = 256;

// ---------------------------------------------------------------------------
// Workgroup shared state
// ---------------------------------------------------------------------------
struct Shared {
  double R[9], t[3];          // current indenter pose
  double pose[7];             // ... as (t, q)
  double iw_lo[3], iw_hi[3];  // indenter world bounding box
  double red[16 * 8];         // per-wave partials
  double bc[8];               // broadcast results
  int count, overflow, flag;
  int pad;
  int rcount[3];              // self-contact region: surface vertices, triangles, edges
  int pad2;
  double qb[7];               // the env's pose at the launch start (motion input)
  T2R_G double* vel;          // this env's velocities (dynamic form)
  double iw, dt;              // inertia weight density / dt^2 (0: quasi-static), time step
  unsigned long long tacc[10];  // wall-clock ticks per phase (thread 0)
};

// Phase timers: thread 0 accumulates wall-clock ticks into S.tacc[k].
__device__ __forceinline__ unsigned long long tick() { return wall_clock64(); }
__device__ __forceinline__ void tock(Shared& S, int k, unsigned long long t0) {
  if (threadIdx.x == 0) S.tacc[k] += wall_clock64() - t0;
}

// LDS of the element passes (staged tile) and, between them, of the pair
// passes (slot positions and sums).
union Tile {
  struct {
    double x[3][kTileVerts];
    double p[3][kTileVerts];
    double g[3][kTileVerts];
    double d[3][kTileVerts];
  };
  struct {                     // curvature pass, mixed precision: x and p rounded to float
    float fx[3][kTileVerts];
    float fp[3][kTileVerts];
  };
  struct {
    double gx[3][kGelSlots];   // gel slot positions
    double gq[3][kGelSlots];   // gradient sums (eval) or p (curvature, CCD)
    double gd[3][kGelSlots];   // diagonal sums (eval)
    double pn[kGelSlots];      // |p|^2 (trial evaluations)
    double iy[3][kIndSlots];   // indenter slot positions, world frame
  };
};

// Block-wide reduction of NS sums followed by NM maxima (values in v[0..NS+NM)).
// Every thread receives the results in v.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce(double* v, Shared& S) {
  constexpr int N = NS + NM;
  static_assert(N <= 8, "block_reduce: at most 8 values (8 slots per wave in Shared::red)");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double a = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double b = __shfl_xor(a, o, 64);
      a = (i < NS) ? a + b : fmax(a, b);
    }
    v[i] = a;
  }
  __syncthreads();  // previous readers of S.red / S.bc are done
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) S.red[wave * 8 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int i = threadIdx.x;
    double a = S.red[i];
    for (int w = 1; w < nw; ++w) a = (i < NS) ? a + S.red[w * 8 + i] : fmax(a, S.red[w * 8 + i]);
    S.bc[i] = a;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = S.bc[i];
}

__device__ __forceinline__ double block_min(double v, Shared& S) {
  double a = -v;
  block_reduce<0, 1>(&a, S);
  return -a;
}

// ---------------------------------------------------------------------------
// Pose helpers (thread 0 writes S)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void quat_to_R(const double q_in[4], double R[9]) {
  const double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
  const double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Pose at tau between p0 and p1: translation linear, rotation by slerp.
__device__ __forceinline__ void interp_pose(const double p0[7], const double p1[7], double tau, double out[7]) {
  #pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = (1.0 - tau) * p0[i] + tau * p1[i];
  double q0[4], q1[4];
  double n0 = 0, n1 = 0;
  #pragma unroll
  for (int i = 0; i < 4; ++i) { q0[i] = p0[3 + i]; q1[i] = p1[3 + i]; n0 += q0[i] * q0[i]; n1 += q1[i] * q1[i]; }
  n0 = sqrt(n0); n1 = sqrt(n1);
  double c = 0;
  #pragma unroll
  for (int i = 0; i < 4; ++i) { q0[i] /= n0; q1[i] /= n1; c += q0[i] * q1[i]; }
  if (c < 0) { for (int i = 0; i < 4; ++i) q1[i] = -q1[i]; c = -c; }
  c = fmin(c, 1.0);
  const double th = acos(c);
  double a, b;
  if (th < 1e-12) { a = 1.0 - tau; b = tau; }
  else { const double s = sin(th); a = sin((1.0 - tau) * th) / s; b = sin(tau * th) / s; }
  double n = 0;
  #pragma unroll
  for (int i = 0; i < 4; ++i) { out[3 + i] = a * q0[i] + b * q1[i]; n += out[3 + i] * out[3 + i]; }
  n = sqrt(n);
  #pragma unroll
  for (int i = 0; i < 4; ++i) out[3 + i] /= n;
}

// Quaternion product a b (w, x, y, z).
__device__ __forceinline__ void quat_mul(const double a[4], const double b[4], double o[4]) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// Unit quaternion of the rotation by the rotation vector w: exp([w]x).
__device__ __forceinline__ void quat_exp(const double w[3], double q[4]) {
  const double a = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double s = a > 1e-12 ? sin(0.5 * a) / a : 0.5 - a * a / 48.0;
  q[0] = cos(0.5 * a);
  q[1] = s * w[0];
  q[2] = s * w[1];
  q[3] = s * w[2];
}

// A pose moved rigidly by (dt, dw): every indenter point R y + t becomes
// exp([dw]x) R y + t + dt, i.e. q <- exp(dw) q (normalised), t <- t + dt.
__device__ __forceinline__ void move_pose(const double in[7], const double dt[3], const double dw[3],
                                          double out[7]) {
  double qn = 0.0;
  #pragma unroll
  for (int i = 3; i < 7; ++i) qn += in[i] * in[i];
  qn = sqrt(qn);
  const double q[4] = {in[3] / qn, in[4] / qn, in[5] / qn, in[6] / qn};
  double e[4], r[4];
  quat_exp(dw, e);
  quat_mul(e, q, r);
  #pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = in[i] + dt[i];
  #pragma unroll
  for (int i = 0; i < 4; ++i) out[3 + i] = r[i];
}

// Rotation vector of the shortest rotation q1 q0^-1 (unit or not).
__device__ __forceinline__ void quat_log_rel(const double q0_in[4], const double q1_in[4], double w[3]) {
  double n0 = 0.0, n1 = 0.0;
  #pragma unroll
  for (int i = 0; i < 4; ++i) { n0 += q0_in[i] * q0_in[i]; n1 += q1_in[i] * q1_in[i]; }
  n0 = sqrt(n0); n1 = sqrt(n1);
  const double c0[4] = {q0_in[0] / n0, -q0_in[1] / n0, -q0_in[2] / n0, -q0_in[3] / n0};
  const double q1[4] = {q1_in[0] / n1, q1_in[1] / n1, q1_in[2] / n1, q1_in[3] / n1};
  double d[4];
  quat_mul(q1, c0, d);
  if (d[0] < 0.0) for (int i = 0; i < 4; ++i) d[i] = -d[i];
  const double s = sqrt(d[1] * d[1] + d[2] * d[2] + d[3] * d[3]);
  const double ang = 2.0 * atan2(s, d[0]);
  const double f = s > 1e-300 ? ang / s : 2.0;
  #pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = f * d[1 + i];
}

// Target pose of load step k (0-based) of a launch of n load steps: the
// caller's pose (moved by the env's rigid offset, if one is set), or the pose
// reached after (k + 1) / n of the launch's motion from the launch-start pose qb.
__device__ __forceinline__ void target_pose(const StepParams& P, const EnvDev& E, int e, int k,
                                            const double qb[7], double q1[7]) {
  if (P.motion_mode == 0) {
    double q[7];
    #pragma unroll
    for (int i = 0; i < 7; ++i) q[i] = P.pose_in[((long long)k * P.n_env + e) * 7 + i];
    if (E.has_off) move_pose(q, E.off, E.off + 3, q1);
    else
      #pragma unroll
      for (int i = 0; i < 7; ++i) q1[i] = q[i];
    return;
  }
  double dt[3], dw[3];
  if (P.motion_mode == 1) {
    #pragma unroll
    for (int i = 0; i < 3; ++i) {
      dt[i] = P.motion_in[6 * e + i] * P.motion_dt;
      dw[i] = P.motion_in[6 * e + 3 + i] * P.motion_dt;
    }
  } else {
    const T2R_G double* a = P.motion_in + 7 * e;
    const T2R_G double* b = P.motion_in2 + 7 * e;
    const double qa[4] = {a[3], a[4], a[5], a[6]}, qbb[4] = {b[3], b[4], b[5], b[6]};
    #pragma unroll
    for (int i = 0; i < 3; ++i) dt[i] = b[i] - a[i];
    quat_log_rel(qa, qbb, dw);
  }
  const double f = (double)(k + 1) / (double)P.n_steps;
  #pragma unroll
  for (int i = 0; i < 3; ++i) { dt[i] *= f; dw[i] *= f; }
  move_pose(qb, dt, dw, q1);
}

__device__ __forceinline__ void set_pose(Shared& S, const IndDev& I, const double pose[7]) {
  for (int i = 0; i < 7; ++i) S.pose[i] = pose[i];
  quat_to_R(pose + 3, S.R);
  #pragma unroll
  for (int i = 0; i < 3; ++i) S.t[i] = pose[i];
  // world box of the local box
  double c[3], h[3];
  #pragma unroll
  for (int i = 0; i < 3; ++i) { c[i] = 0.5 * (I.box_lo[i] + I.box_hi[i]); h[i] = 0.5 * (I.box_hi[i] - I.box_lo[i]); }
  #pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double cw = S.R[a * 3 + 0] * c[0] + S.R[a * 3 + 1] * c[1] + S.R[a * 3 + 2] * c[2] + S.t[a];
    const double hw = fabs(S.R[a * 3 + 0]) * h[0] + fabs(S.R[a * 3 + 1]) * h[1] + fabs(S.R[a * 3 + 2]) * h[2];
    S.iw_lo[a] = cw - hw;
    S.iw_hi[a] = cw + hw;
  }
}

__device__ __forceinline__ void ind_world(const Shared& S, const IndDev& I, int j, double y[3]) {
  const double a = I.Y[j], b = I.Y[I.n_v + j], c = I.Y[2 * I.n_v + j];
  #pragma unroll
  for (int r = 0; r < 3; ++r) y[r] = S.R[r * 3 + 0] * a + S.R[r * 3 + 1] * b + S.R[r * 3 + 2] * c + S.t[r];
}

// ---------------------------------------------------------------------------
// Env view: pointers of one env's state
// ---------------------------------------------------------------------------
struct View {
  const T2R_G GelDev* G;
  const T2R_G IndDev* I;
  const T2R_G EnvDev* E;
  T2R_G double* x;
  T2R_G double* xprev;
  T2R_G double* g0;
  T2R_G double* g1;
  T2R_G double* diag;
  T2R_G double* p;
  T2R_G int2* pairs;
  T2R_G double* pd;      // distance of each candidate pair at the current x
  T2R_G int2* outer;     // coarse candidates within the outer radius
  T2R_G FricPair* fric;
  T2R_G int* vmap;
  T2R_G int* imap;
  T2R_G uint64_t* oslot;
  T2R_G uint64_t* pslot;
  T2R_G int* slot_v;
  T2R_G int* islot_v;
  int npairs, nfric, nouter;
  int nslots, nislots, slots_ok;
  int mixed;
  int moll;              // edge-edge mollifier on
  int det;               // deterministic order: summing passes and list builds on one thread
  int selfc;             // self-contact pairs (gel surface vs gel surface)
};

// Item loops of the passes that sum into shared per-vertex slots or append to
// lists: block-strided, or in deterministic mode all on thread 0 in index
// order (every sum and every list then has a fixed order, so results repeat
// bit for bit).
__device__ __forceinline__ unsigned item_first(const View& V) {
  return V.det ? (threadIdx.x == 0 ? 0u : 0x7fffffffu) : threadIdx.x;
}
__device__ __forceinline__ unsigned item_step(const View& V) { return V.det ? 1u : blockDim.x; }

// ---------------------------------------------------------------------------
// Element passes over LDS-staged tiles
//
// A tile is a contiguous run of tets whose vertices (<= kTileVerts, local ids
// in tet_local) are staged in LDS. Each thread owns up to kSlots vertex slots
// of every tile; the global loads for the next tile's slots are issued into
// registers before the current tile's tets are computed, so HBM/L2 latency
// overlaps the arithmetic, and the per-tet inputs (local ids, Dm^-1, volume)
// are likewise loaded one tet ahead.
// ---------------------------------------------------------------------------
constexpr int kSlots = kTileVerts / 256;  // vertex slots per thread (blocks of >= 256 threads)

template <bool MIXED>
struct TetIn {
  using R = typename std::conditional<MIXED, float, double>::type;
  uint64_t loc;
  R Dm[9];
  R vol;
};

template <bool MIXED>
__device__ __forceinline__ void load_tet(const GelDev& G, int e, TetIn<MIXED>& t) {
  t.loc = G.tet_local[e];
  if constexpr (MIXED) {
#pragma unroll
    for (int k = 0; k < 9; ++k) t.Dm[k] = G.Dinv32[k * G.n_t + e];
    t.vol = G.vol32[e];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) t.Dm[k] = G.Dinv[k * G.n_t + e];
    t.vol = G.vol[e];
  }
}

__device__ __forceinline__ void tet_ids(uint64_t loc, int l[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) l[k] = (int)((loc >> (16 * k)) & 0xffff);
}

// Vertex ids and flags of one thread's slots of a tile. Loads are clamped to
// valid addresses so that they issue unconditionally (exact wait counts); a
// slot past the tile's vertices, or of a tile past the last, has fl = -1.
struct SlotIdx {
  int v[kSlots];
  int fl[kSlots];
};

__device__ __forceinline__ void fetch_idx(const GelDev& G, int tile, SlotIdx& I) {
  const bool live = tile < G.n_tiles;
  const int t = live ? tile : G.n_tiles - 1;
  const int v0 = G.tile_vstart[t], ntv = G.tile_vstart[t + 1] - v0;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int i = threadIdx.x + s * blockDim.x;
    const int j = v0 + min(i, ntv - 1);
    I.v[s] = G.tile_verts[j];
    const int f = G.tile_flags[j];
    I.fl[s] = (live && i < ntv) ? f : -1;
  }
}

// First tet of this thread at or after tile `tile` (clamped to a valid id).
__device__ __forceinline__ int first_tet(const GelDev& G, int tile) {
  const int t = min(tile, G.n_tiles - 1);
  return min(G.tile_tet[t] + (int)threadIdx.x, G.n_t - 1);
}

// Evaluates sum V psi, the gradient and diag(H) of the elastic term at
// x + alpha p (p not null) into gout/dout ([3][n_v]). Returns energy (thread
// partial) and clears `feasible` on an inverted tet. Fixed vertices get g = 0,
// diag = 1.
//
// Pipeline per tile k: the positions of tile k+1, the slot ids of tile k+2,
// the earlier partial sums of tile k's shared vertices and each thread's next
// tet are loaded into registers while tile k's tets are computed from LDS.
template <bool MIXED>
__device__ __forceinline__ double elem_eval_impl(const View& V, const double* x, const double* p, double alpha,
                                                 double* gout, double* dout, Tile& T, int& feasible) {
  const GelDev& G = *V.G;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const int B = blockDim.x;
  const int NT = G.n_tiles;
  double energy = 0.0;
  if (NT == 0) return energy;
  // every g/d slot is zero between tiles: each flush clears what it read
  for (int i = threadIdx.x; i < kTileVerts; i += B) {
#pragma unroll
    for (int c = 0; c < 3; ++c) { T.g[c][i] = 0.0; T.d[c][i] = 0.0; }
  }
  SlotIdx cur, nxt;
  fetch_idx(G, 0, cur);
  fetch_idx(G, 1, nxt);
  double a[kSlots][3];
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) a[s][c] = fma(alpha, p[c * nv + cur.v[s]], x[c * nv + cur.v[s]]);
  TetIn<MIXED> tc;
  load_tet<MIXED>(G, first_tet(G, 0), tc);
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
    if (cur.fl[s] >= 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) T.x[c][threadIdx.x + s * B] = a[s][c];
  __syncthreads();
  for (int tile = 0; tile < NT; ++tile) {
    const int t0 = G.tile_tet[tile], t1 = G.tile_tet[tile + 1];
    double og[kSlots][3], od[kSlots][3];
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        og[s][c] = gout[c * nv + cur.v[s]];
        od[s][c] = dout[c * nv + cur.v[s]];
      }
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) a[s][c] = fma(alpha, p[c * nv + nxt.v[s]], x[c * nv + nxt.v[s]]);
    SlotIdx nn;
    fetch_idx(G, tile + 2, nn);
    // deterministic mode: the tile's tets on thread 0, in tile order (its next
    // tet is then e + 1, and after the tile the first tet of the next one)
    const int e_first = V.det ? (threadIdx.x == 0 ? t0 : t1) : t0 + (int)threadIdx.x;
    const int e_step = V.det ? 1 : B;
    for (int e = e_first; e < t1; e += e_step) {
      TetIn<MIXED> tn;
      const int en = (e + e_step < t1) ? e + e_step : first_tet(G, tile + 1);
      load_tet<MIXED>(G, en, tn);
      int l[4];
      tet_ids(tc.loc, l);
      double Ds[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) Ds[r * 3 + k] = T.x[r][l[k + 1]] - T.x[r][l[0]];
      double ed = 0.0;
      bool ok;
      if constexpr (MIXED) {
        ok = tet_grad_diag_mixed(Ds, tc.Dm, tc.vol, E.mu, E.lam, ed,
                                 [&](int k, int c, auto gv, auto dv) {
                                   atomicAdd(&T.g[c][l[k]], (double)gv);
                                   atomicAdd(&T.d[c][l[k]], (double)dv);
                                 });
      } else {
        ok = tet_grad_diag64(Ds, tc.Dm, tc.vol, E.mu, E.lam, ed,
                             [&](int k, int c, double gv, double dv) {
                               atomicAdd(&T.g[c][l[k]], gv);
                               atomicAdd(&T.d[c][l[k]], dv);
                             });
      }
      if (ok) energy += ed;
      else feasible = 0;
      tc = tn;
    }
    // a thread without a tet here fetches its first tet of the next tile
    if (e_first >= t1) load_tet<MIXED>(G, first_tet(G, tile + 1), tc);
    __syncthreads();
    // flush this tile's slots, clear them, stage the next tile's positions
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const int i = threadIdx.x + s * B;
      if (cur.fl[s] >= 0) {
        const int v = cur.v[s];
        const bool first = cur.fl[s] & kFirstTouch;
        const bool fixed = cur.fl[s] & kFixedLast;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double gv = T.g[c][i], dv = T.d[c][i];
          if (!first) { gv += og[s][c]; dv += od[s][c]; }
          T.g[c][i] = 0.0;
          T.d[c][i] = 0.0;
          if (fixed) { gv = 0.0; dv = 1.0; }
          gout[c * nv + v] = gv;
          dout[c * nv + v] = dv;
        }
      }
      if (nxt.fl[s] >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) T.x[c][i] = a[s][c];
      }
    }
    cur = nxt;
    nxt = nn;
    __syncthreads();
  }
  return energy;
}

__device__ __forceinline__ double elem_eval(const View& V, const double* x, const double* p, double alpha,
                                            double* gout, double* dout, Tile& T, int& feasible) {
  return V.mixed ? elem_eval_impl<true>(V, x, p, alpha, gout, dout, T, feasible)
                 : elem_eval_impl<false>(V, x, p, alpha, gout, dout, T, feasible);
}

// Stages one vertex coordinate of x and p for the curvature pass: as float in
// mixed precision (p^T H p only sets the trial step; float positions of a
// ~10 mm gel are within 1e-6 mm), else as double.
template <bool MIXED>
__device__ __forceinline__ void stage_xp(Tile& T, int c, int i, double xv, double pv) {
  if constexpr (MIXED) {
    T.fx[c][i] = (float)xv;
    T.fp[c][i] = (float)pv;
  } else {
    T.x[c][i] = xv;
    T.p[c][i] = pv;
  }
}

// p^T H_elastic p at x (thread partial); same pipeline as the eval pass.
template <bool MIXED>
__device__ __forceinline__ double elem_curv_impl(const View& V, const double* x, const double* p, Tile& T) {
  const GelDev& G = *V.G;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const int B = blockDim.x;
  const int NT = G.n_tiles;
  using Rl = typename TetIn<MIXED>::R;
  double curv = 0.0;
  if (NT == 0) return curv;
  SlotIdx cur, nxt;
  fetch_idx(G, 0, cur);
  fetch_idx(G, 1, nxt);
  double a[kSlots][3], b[kSlots][3];
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a[s][c] = x[c * nv + cur.v[s]];
      b[s][c] = p[c * nv + cur.v[s]];
    }
  TetIn<MIXED> tc, tc1;  // tc1: the second tet of a pair (mixed precision)
  load_tet<MIXED>(G, first_tet(G, 0), tc);
  if constexpr (MIXED) load_tet<MIXED>(G, min(first_tet(G, 0) + B, G.n_t - 1), tc1);
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
    if (cur.fl[s] >= 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) stage_xp<MIXED>(T, c, threadIdx.x + s * B, a[s][c], b[s][c]);
  __syncthreads();
  for (int tile = 0; tile < NT; ++tile) {
    const int t0 = G.tile_tet[tile], t1 = G.tile_tet[tile + 1];
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a[s][c] = x[c * nv + nxt.v[s]];
        b[s][c] = p[c * nv + nxt.v[s]];
      }
    SlotIdx nn;
    fetch_idx(G, tile + 2, nn);
    if constexpr (MIXED) {
      // a thread's tets of the tile in pairs (e, e + B): both tets' LDS reads and
      // FP32 arithmetic sit in one block, so the two chains hide each other's
      // latency; the next pair's tet data is in flight meanwhile
      for (int e = t0 + threadIdx.x; e < t1; e += 2 * B) {
        const bool two = e + B < t1;
        const int en0 = (e + 2 * B < t1) ? e + 2 * B : first_tet(G, tile + 1);
        TetIn<MIXED> tn, tn1;
        load_tet<MIXED>(G, en0, tn);
        load_tet<MIXED>(G, min(en0 + B, G.n_t - 1), tn1);
        int la[4], lb[4];
        tet_ids(tc.loc, la);
        tet_ids(tc1.loc, lb);
        float DsA[9], dDsA[9], DsB[9], dDsB[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            DsA[r * 3 + k] = T.fx[r][la[k + 1]] - T.fx[r][la[0]];
            dDsA[r * 3 + k] = T.fp[r][la[k + 1]] - T.fp[r][la[0]];
            DsB[r * 3 + k] = T.fx[r][lb[k + 1]] - T.fx[r][lb[0]];
            dDsB[r * 3 + k] = T.fp[r][lb[k + 1]] - T.fp[r][lb[0]];
          }
        const float JA = DsA[0] * (DsA[4] * DsA[8] - DsA[5] * DsA[7]) - DsA[1] * (DsA[3] * DsA[8] - DsA[5] * DsA[6]) +
                         DsA[2] * (DsA[3] * DsA[7] - DsA[4] * DsA[6]);
        const float JB = DsB[0] * (DsB[4] * DsB[8] - DsB[5] * DsB[7]) - DsB[1] * (DsB[3] * DsB[8] - DsB[5] * DsB[6]) +
                         DsB[2] * (DsB[3] * DsB[7] - DsB[4] * DsB[6]);
        // det Ds at rest = 6 V; a tet squashed below kMixedMinJ takes FP64 from the
        // global positions (FP32 cofactors lose the sign of det F as J -> 0)
        const bool okA = JA > (float)kMixedMinJ * 6.0f * tc.vol;
        const bool okB = !two || JB > (float)kMixedMinJ * 6.0f * tc1.vol;
        if (okA && okB) {
          const float cA = tet_curvature<float>(DsA, dDsA, tc.Dm, tc.vol, (float)E.mu, (float)E.lam);
          const float cB = tet_curvature<float>(DsB, dDsB, tc1.Dm, tc1.vol, (float)E.mu, (float)E.lam);
          curv += (double)cA + (two ? (double)cB : 0.0);
        } else {
          auto slow = [&](const TetIn<MIXED>& t, int et, const float* Ds, const float* dDs, bool ok) {
            if (ok) return (double)tet_curvature<float>(Ds, dDs, t.Dm, t.vol, (float)E.mu, (float)E.lam);
            double Ds64[9], dDs64[9], Dm64[9];
            int gv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) gv[k] = G.tet[k * G.n_t + et];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                Ds64[r * 3 + k] = x[r * nv + gv[k + 1]] - x[r * nv + gv[0]];
                dDs64[r * 3 + k] = p[r * nv + gv[k + 1]] - p[r * nv + gv[0]];
              }
#pragma unroll
            for (int k = 0; k < 9; ++k) Dm64[k] = (double)t.Dm[k];
            return tet_curvature<double>(Ds64, dDs64, Dm64, (double)t.vol, E.mu, E.lam);
          };
          curv += slow(tc, e, DsA, dDsA, okA);
          if (two) curv += slow(tc1, e + B, DsB, dDsB, JB > (float)kMixedMinJ * 6.0f * tc1.vol);
        }
        tc = tn;
        tc1 = tn1;
      }
    } else {
      for (int e = t0 + threadIdx.x; e < t1; e += B) {
        TetIn<MIXED> tn;
        const int en = (e + B < t1) ? e + B : first_tet(G, tile + 1);
        load_tet<MIXED>(G, en, tn);
        int l[4];
        tet_ids(tc.loc, l);
        Rl Ds[9], dDs[9];
  #pragma unroll
        for (int r = 0; r < 3; ++r)
  #pragma unroll
          for (int k = 0; k < 3; ++k) {
            if constexpr (MIXED) {
              Ds[r * 3 + k] = T.fx[r][l[k + 1]] - T.fx[r][l[0]];
              dDs[r * 3 + k] = T.fp[r][l[k + 1]] - T.fp[r][l[0]];
            } else {
              Ds[r * 3 + k] = T.x[r][l[k + 1]] - T.x[r][l[0]];
              dDs[r * 3 + k] = T.p[r][l[k + 1]] - T.p[r][l[0]];
            }
          }
        if constexpr (MIXED) {
          // a tet squashed below kMixedMinJ: FP64 from the global positions
          // (FP32 cofactors lose the sign of det F as J -> 0)
          const float J32 = Ds[0] * (Ds[4] * Ds[8] - Ds[5] * Ds[7]) - Ds[1] * (Ds[3] * Ds[8] - Ds[5] * Ds[6]) +
                            Ds[2] * (Ds[3] * Ds[7] - Ds[4] * Ds[6]);
          const float Jref = 6.0f * tc.vol;  // det Ds at rest = 6 V
          if (!(J32 > (float)kMixedMinJ * Jref)) {
            double Ds64[9], dDs64[9], Dm64[9];
            int gv[4];
  #pragma unroll
            for (int k = 0; k < 4; ++k) gv[k] = G.tet[k * G.n_t + e];
  #pragma unroll
            for (int r = 0; r < 3; ++r)
  #pragma unroll
              for (int k = 0; k < 3; ++k) {
                Ds64[r * 3 + k] = x[r * nv + gv[k + 1]] - x[r * nv + gv[0]];
                dDs64[r * 3 + k] = p[r * nv + gv[k + 1]] - p[r * nv + gv[0]];
              }
  #pragma unroll
            for (int k = 0; k < 9; ++k) Dm64[k] = (double)tc.Dm[k];
            curv += tet_curvature<double>(Ds64, dDs64, Dm64, (double)tc.vol, E.mu, E.lam);
          } else {
            curv += (double)tet_curvature<Rl>(Ds, dDs, tc.Dm, tc.vol, (Rl)E.mu, (Rl)E.lam);
          }
        } else {
          curv += (double)tet_curvature<Rl>(Ds, dDs, tc.Dm, tc.vol, (Rl)E.mu, (Rl)E.lam);
        }
        tc = tn;
      }
    }
    if (t0 + (int)threadIdx.x >= t1) {
      load_tet<MIXED>(G, first_tet(G, tile + 1), tc);
      if constexpr (MIXED) load_tet<MIXED>(G, min(first_tet(G, tile + 1) + B, G.n_t - 1), tc1);
    }
    __syncthreads();
    if (tile + 1 < NT) {
#pragma unroll
      for (int s = 0; s < kSlots; ++s)
        if (nxt.fl[s] >= 0)
#pragma unroll
          for (int c = 0; c < 3; ++c) stage_xp<MIXED>(T, c, threadIdx.x + s * B, a[s][c], b[s][c]);
      __syncthreads();
    }
    cur = nxt;
    nxt = nn;
  }
  return curv;
}

__device__ __forceinline__ double elem_curv(const View& V, const double* x, const double* p, Tile& T) {
  return V.mixed ? elem_curv_impl<true>(V, x, p, T) : elem_curv_impl<false>(V, x, p, T);
}

// ---------------------------------------------------------------------------
// Contact pairs
//
// With contact slots (V.slots_ok) a pair pass first stages the positions of the
// listed pairs' gel vertices and the world positions of their indenter
// vertices in LDS; each pair is then one 8-byte record read, LDS reads and LDS
// atomics, and the gradient sums reach global memory once per gel vertex.
// Without slots (too many vertices near the indenter) the same passes gather
// from global memory and add with global atomics.
// ---------------------------------------------------------------------------
struct PairPts {
  double z[4][3];
  int gid[4];      // gel point: slot (LDS path) or vertex id (global path); -1: indenter point
  int kind;
};

__device__ __forceinline__ int rec_kind(uint64_t r) { return (int)(r >> (4 * kRecBits)) & 7; }
__device__ __forceinline__ int rec_slot(uint64_t r, int k) {
  return (int)(r >> (kRecBits * k)) & ((1 << kRecBits) - 1);
}
// Point k of a pair is a gel point: VF (gel vertex, indenter triangle),
// FV (indenter vertex, gel triangle), EE (gel edge, indenter edge); every point
// of the self-contact kinds GVF (gel vertex, gel triangle) and GEE (two gel edges).
__device__ __forceinline__ bool point_is_gel(int kind, int k) {
  return kind >= kGVF ? true : (kind == kVF ? k == 0 : (kind == kFV ? k > 0 : k < 2));
}

// Bound on how fast a pair's distance can shrink when its gel points move with
// squared speeds s[k] (0 for indenter points): the largest gel speed, or for a
// self-contact pair, whose two primitives both move, the sum of each side's.
__device__ __forceinline__ double closing_rate(int selfc, int kind, const double s[4]) {
  if (selfc && kind == kGVF) return sqrt(s[0]) + sqrt(fmax(fmax(s[1], s[2]), s[3]));
  if (selfc && kind == kGEE) return sqrt(fmax(s[0], s[1])) + sqrt(fmax(s[2], s[3]));
  return sqrt(fmax(fmax(s[0], s[1]), fmax(s[2], s[3])));
}

// Vertex ids of the four points of pair `pr` (gel ids where point_is_gel).
__device__ __forceinline__ void pair_point_ids(const GelDev& G, const IndDev& I, int2 pr, int id[4]) {
  const int kind = (int)((unsigned)pr.x >> kKindShift);
  const int gp = pr.x & kPrimMask, ip = pr.y;
  if (kind == kVF) {
    id[0] = gp;
    id[1] = I.tri[ip]; id[2] = I.tri[I.n_f + ip]; id[3] = I.tri[2 * I.n_f + ip];
  } else if (kind == kFV) {
    id[0] = ip;
    id[1] = G.surf_f[gp]; id[2] = G.surf_f[G.n_sf + gp]; id[3] = G.surf_f[2 * G.n_sf + gp];
  } else if (kind == kEE) {
    id[0] = G.surf_e[gp]; id[1] = G.surf_e[G.n_se + gp];
    id[2] = I.edge[ip]; id[3] = I.edge[I.n_e + ip];
  } else if (kind == kGVF) {
    id[0] = gp;
    id[1] = G.surf_f[ip]; id[2] = G.surf_f[G.n_sf + ip]; id[3] = G.surf_f[2 * G.n_sf + ip];
  } else {
    id[0] = G.surf_e[gp]; id[1] = G.surf_e[G.n_se + gp];
    id[2] = G.surf_e[ip]; id[3] = G.surf_e[G.n_se + ip];
  }
}

// Global path: gathers the four points of pair `pr`; gel points at x + alpha p.
__device__ __forceinline__ void load_pair(const View& V, const Shared& S, int2 pr, const double* x,
                                          const double* p, double alpha, PairPts& P) {
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const int nv = G.n_v;
  const int kind = (int)((unsigned)pr.x >> kKindShift);
  int id[4];
  pair_point_ids(G, I, pr, id);
  P.kind = kind;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (point_is_gel(kind, k)) {
      P.gid[k] = id[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double xv = x[c * nv + id[k]];
        P.z[k][c] = p ? fma(alpha, p[c * nv + id[k]], xv) : xv;
      }
    } else {
      P.gid[k] = -1;
      ind_world(S, I, id[k], P.z[k]);
    }
  }
}

// LDS path: the four points of a pair record from the staged slots.
__device__ __forceinline__ void load_pair_lds(const Tile& T, uint64_t rec, PairPts& P) {
  const int kind = rec_kind(rec);
  P.kind = kind;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = rec_slot(rec, k);
    if (point_is_gel(kind, k)) {
      P.gid[k] = q;
#pragma unroll
      for (int c = 0; c < 3; ++c) P.z[k][c] = T.gx[c][q];
    } else {
      P.gid[k] = -1;
#pragma unroll
      for (int c = 0; c < 3; ++c) P.z[k][c] = T.iy[c][q];
    }
  }
}

template <bool LDS>
__device__ __forceinline__ void get_pair(const View& V, const Shared& S, const Tile& T, int2 pr, uint64_t rec,
                                         const double* x, const double* p, double alpha, PairPts& P) {
  if constexpr (LDS) load_pair_lds(T, rec, P);
  else load_pair(V, S, pr, x, p, alpha, P);
}

__device__ __forceinline__ void classify(const PairPts& P, Feature& f) {
  if (P.kind == kEE || P.kind == kGEE) classify_ee(P.z[0], P.z[1], P.z[2], P.z[3], f);
  else classify_pt(P.z[0], P.z[1], P.z[2], P.z[3], f);
}

__device__ __forceinline__ double pair_distance(const PairPts& P, const Feature& f, double r[3]) {
  #pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = f.c[0] * P.z[0][c] + f.c[1] * P.z[1][c] + f.c[2] * P.z[2][c] + f.c[3] * P.z[3][c];
  return sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

// Edge-edge mollifier of pair P (edge vectors a = z1 - z0 of the gel edge and
// b = z3 - z2 of the indenter edge): false unless the option is on, P is an
// edge-edge pair and c = |a x b|^2 lies below e = kEdgeMollRel |a_rest|^2
// |b_rest|^2 (rest gel positions, local indenter positions). With c as a
// function of the four points: dc/dz1 = -dc/dz0 = ga = 2 (|b|^2 a - (a.b) b),
// dc/dz3 = -dc/dz2 = gb = 2 (|a|^2 b - (a.b) a), d2c/da2 = 2 (|b|^2 I - b b^T)
// and d2c/da db = 4 a b^T - 2 b a^T - 2 (a.b) I.
struct EdgeMoll {
  double m, m1, m2;       // m(c), m'(c), m''(c)
  double a[3], b[3];
  double aa, bb, ab;
};

template <bool LDS>
__device__ __forceinline__ bool edge_moll(const View& V, int2 pr, uint64_t rec, const PairPts& P, EdgeMoll& M) {
  if (!V.moll || (P.kind != kEE && P.kind != kGEE)) return false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    M.a[c] = P.z[1][c] - P.z[0][c];
    M.b[c] = P.z[3][c] - P.z[2][c];
  }
  const double w[3] = {M.a[1] * M.b[2] - M.a[2] * M.b[1], M.a[2] * M.b[0] - M.a[0] * M.b[2],
                       M.a[0] * M.b[1] - M.a[1] * M.b[0]};
  const double cx = dot3(w, w);
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  int id[4];
  const bool self = P.kind == kGEE;  // second edge on the gel too
  if constexpr (LDS) {
    id[0] = V.slot_v[rec_slot(rec, 0)];
    id[1] = V.slot_v[rec_slot(rec, 1)];
    id[2] = self ? V.slot_v[rec_slot(rec, 2)] : V.islot_v[rec_slot(rec, 2)];
    id[3] = self ? V.slot_v[rec_slot(rec, 3)] : V.islot_v[rec_slot(rec, 3)];
  } else {
    pair_point_ids(G, I, pr, id);
  }
  double ar = 0.0, br = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double u = G.X[c * G.n_v + id[1]] - G.X[c * G.n_v + id[0]];
    const double v = self ? G.X[c * G.n_v + id[3]] - G.X[c * G.n_v + id[2]]
                          : I.Y[c * I.n_v + id[3]] - I.Y[c * I.n_v + id[2]];
    ar += u * u;
    br += v * v;
  }
  const double e = kEdgeMollRel * ar * br;
  if (!(cx < e)) return false;
  edge_mollifier3(cx, e, M.m, M.m1, M.m2);
  M.aa = dot3(M.a, M.a);
  M.bb = dot3(M.b, M.b);
  M.ab = dot3(M.a, M.b);
  return true;
}

// Stages the slot points of the env for a pair pass. what: 0 positions x;
// 1 positions x and p (in gq); 2 positions x + alpha p, |p|^2 (in pn), cleared
// gradient/diagonal sums (p not null for 1 and 2). The indenter points are
// placed at the current pose. Starts and ends with a barrier.
__device__ __forceinline__ void stage_points(const View& V, const Shared& S, Tile& T, const double* x,
                                             const double* p, double alpha, int what) {
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const int nv = G.n_v;
  __syncthreads();  // the tile storage may still be read by the previous pass
  for (int i = threadIdx.x; i < V.nslots; i += blockDim.x) {
    const int v = V.slot_v[i];
    double pv2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double xv = x[c * nv + v];
      if (what == 2) {
        const double pv = p[c * nv + v];
        T.gx[c][i] = fma(alpha, pv, xv);
        T.gq[c][i] = 0.0;
        T.gd[c][i] = 0.0;
        pv2 += pv * pv;
      } else {
        T.gx[c][i] = xv;
        if (what == 1) T.gq[c][i] = p[c * nv + v];
      }
    }
    if (what == 2) T.pn[i] = pv2;
  }
  for (int i = threadIdx.x; i < V.nislots; i += blockDim.x) {
    double y[3];
    ind_world(S, I, V.islot_v[i], y);
#pragma unroll
    for (int c = 0; c < 3; ++c) T.iy[c][i] = y[c];
  }
  __syncthreads();
}

// Adds the staged gradient/diagonal sums of the slots to gout/dout (free gel
// vertices only). Starts with a barrier.
__device__ __forceinline__ void flush_slots(const View& V, const Tile& T, double* gout, double* dout) {
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  __syncthreads();
  for (int i = threadIdx.x; i < V.nslots; i += blockDim.x) {
    const int v = V.slot_v[i];
    if (G.fixed[v]) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gout[c * nv + v] += T.gq[c][i];
      dout[c * nv + v] += T.gd[c][i];
    }
  }
}

// Barrier energy, gradient and diag of every candidate pair at x + alpha p.
// For a trial step, a pair whose cached distance minus the largest motion of
// its gel vertices stays >= dhat is inactive (and positive) at the trial point:
// its cache keeps that lower bound and no exact distance is computed.
template <bool LDS>
__device__ __forceinline__ double pairs_eval(const View& V, const Shared& S, Tile& T, const double* x,
                                             const double* p, double alpha, double* gout, double* dout,
                                             int& feasible, int& nactive) {
  const GelDev& G = *V.G;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const double dh = E.dhat, kap = E.kappa;
  double energy = 0.0;
  for (int i = item_first(V); i < V.npairs; i += item_step(V)) {
    int2 pr = make_int2(0, 0);
    uint64_t rec = 0;
    if constexpr (LDS) rec = V.pslot[i];
    else pr = V.pairs[i];
    if (alpha > 0.0) {
      double sk[4] = {0.0, 0.0, 0.0, 0.0};
      int kind;
      if constexpr (LDS) {
        kind = rec_kind(rec);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (point_is_gel(kind, k)) sk[k] = T.pn[rec_slot(rec, k)];
      } else {
        int id[4];
        pair_point_ids(G, *V.I, pr, id);
        kind = (int)((unsigned)pr.x >> kKindShift);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (!point_is_gel(kind, k)) continue;
          double sq = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) { const double pc = p[c * nv + id[k]]; sq += pc * pc; }
          sk[k] = sq;
        }
      }
      const double lb = V.pd[i] - alpha * closing_rate(V.selfc, kind, sk);
      if (lb >= dh) { V.pd[i] = lb; continue; }
    }
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, p, alpha, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    V.pd[i] = d;
    if (!(d > 0.0)) { feasible = 0; continue; }
    if (d >= dh) continue;
    ++nactive;
    double b, b1, b2;
    barrier3(d, dh, b, b1, b2);
    EdgeMoll M;
    const bool mol = edge_moll<LDS>(V, pr, rec, P, M);
    double ga[3] = {0.0, 0.0, 0.0}, gb[3] = {0.0, 0.0, 0.0};
    if (mol) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ga[c] = 2.0 * (M.bb * M.a[c] - M.ab * M.b[c]);
        gb[c] = 2.0 * (M.aa * M.b[c] - M.ab * M.a[c]);
      }
    }
    energy += kap * (mol ? M.m * b : b);
    const double invd = 1.0 / d;
    double n[3] = {r[0] * invd, r[1] * invd, r[2] * invd};
    double D[2][3] = {{0, 0, 0}, {0, 0, 0}};
    #pragma unroll
    for (int w = 0; w < 2; ++w)
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        D[w][c] = cw_of(f, 0, w) * P.z[0][c] + cw_of(f, 1, w) * P.z[1][c] + cw_of(f, 2, w) * P.z[2][c] + cw_of(f, 3, w) * P.z[3][c];
    double Mi[2][2];
    gram_inverse(D, f.k, Mi);
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = P.gid[k];
      if (v < 0) continue;
      if (!LDS && G.fixed[v]) continue;
      const double ci = f.c[k];
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double gi = ci * n[c];
        double u0 = 0.0, u1 = 0.0;
        if (f.k > 0) u0 = cw_of(f, k, 0) * r[c] + ci * D[0][c];
        if (f.k > 1) u1 = cw_of(f, k, 1) * r[c] + ci * D[1][c];
        const double uMu = u0 * (Mi[0][0] * u0 + Mi[0][1] * u1) + u1 * (Mi[1][0] * u0 + Mi[1][1] * u1);
        const double hdd = (ci * ci - uMu) * invd - gi * gi * invd;
        // preconditioner diagonal: the pair's contribution clamped at zero (b' < 0
        // makes it negative in directions tangent to a close contact)
        double gval = kap * b1 * gi, hval = b2 * gi * gi + b1 * hdd;
        if (mol) {  // gel points: the first edge (k = 0, 1), and for a gel-gel pair the second (2, 3)
          const double gc = k == 0 ? -ga[c] : (k == 1 ? ga[c] : (k == 2 ? -gb[c] : gb[c]));
          const double hc = k < 2 ? 2.0 * (M.bb - M.b[c] * M.b[c]) : 2.0 * (M.aa - M.a[c] * M.a[c]);
          gval = kap * (M.m * b1 * gi + M.m1 * b * gc);
          hval = M.m * hval + 2.0 * M.m1 * b1 * gi * gc + M.m2 * b * gc * gc + M.m1 * b * hc;
        }
        const double dval = kap * fmax(0.0, hval);
        if constexpr (LDS) {
          atomicAdd(&T.gq[c][v], gval);
          atomicAdd(&T.gd[c][v], dval);
        } else {
          atomicAdd(&gout[c * nv + v], gval);
          atomicAdd(&dout[c * nv + v], dval);
        }
      }
    }
  }
  return energy;
}

// p^T H_barrier p at x (thread partial). LDS path: gx = x, gq = p.
template <bool LDS>
__device__ __forceinline__ double pairs_curv(const View& V, const Shared& S, const Tile& T, const double* x,
                                             const double* p) {
  const GelDev& G = *V.G;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const double dh = E.dhat, kap = E.kappa;
  double curv = 0.0;
  for (int i = threadIdx.x; i < V.npairs; i += blockDim.x) {
    if (!(V.pd[i] < dh)) continue;  // inactive at x: no barrier curvature
    int2 pr = make_int2(0, 0);
    uint64_t rec = 0;
    if constexpr (LDS) rec = V.pslot[i];
    else pr = V.pairs[i];
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    if (!(d > 0.0) || d >= dh) continue;
    double b, b1, b2;
    barrier3(d, dh, b, b1, b2);
    const double invd = 1.0 / d;
    double n[3] = {r[0] * invd, r[1] * invd, r[2] * invd};
    double D[2][3] = {{0, 0, 0}, {0, 0, 0}};
    #pragma unroll
    for (int w = 0; w < 2; ++w)
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        D[w][c] = cw_of(f, 0, w) * P.z[0][c] + cw_of(f, 1, w) * P.z[1][c] + cw_of(f, 2, w) * P.z[2][c] + cw_of(f, 3, w) * P.z[3][c];
    double Mi[2][2];
    gram_inverse(D, f.k, Mi);
    double q[3] = {0, 0, 0}, vv[2] = {0, 0}, da[3] = {0, 0, 0}, db[3] = {0, 0, 0};
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = P.gid[k];
      if (v < 0) continue;
      double pk[3];
      #pragma unroll
      for (int c = 0; c < 3; ++c) pk[c] = LDS ? T.gq[c][v] : p[c * nv + v];  // p = 0 on fixed vertices
      #pragma unroll
      for (int c = 0; c < 3; ++c) q[c] += f.c[k] * pk[c];
      // p_1 - p_0 and p_3 - p_2 of an edge-edge pair (indenter points: p = 0)
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (k < 2) da[c] += k == 0 ? -pk[c] : pk[c];
        else db[c] += k == 2 ? -pk[c] : pk[c];
      }
      const double rp = dot3(r, pk);
      #pragma unroll
      for (int w = 0; w < 2; ++w) if (w < f.k) vv[w] += cw_of(f, k, w) * rp + f.c[k] * dot3(D[w], pk);
    }
    const double nq = dot3(n, q);
    const double vMv = vv[0] * (Mi[0][0] * vv[0] + Mi[0][1] * vv[1]) + vv[1] * (Mi[1][0] * vv[0] + Mi[1][1] * vv[1]);
    const double pHp = (dot3(q, q) - vMv) * invd - nq * nq * invd;
    double cv = b2 * nq * nq + b1 * pHp;
    EdgeMoll M;
    if (edge_moll<LDS>(V, pr, rec, P, M)) {
      const double ad = dot3(M.a, da), bd = dot3(M.b, da), ae = dot3(M.a, db), be = dot3(M.b, db);
      const double cp = 2.0 * (M.bb * ad - M.ab * bd) + 2.0 * (M.aa * be - M.ab * ae);   // grad c . p
      const double pHc = 2.0 * (M.bb * dot3(da, da) - bd * bd) + 2.0 * (M.aa * dot3(db, db) - ae * ae) +
                         2.0 * (4.0 * ad * be - 2.0 * bd * ae - 2.0 * M.ab * dot3(da, db));   // p^T (d2c) p
      cv = M.m * cv + 2.0 * M.m1 * b1 * nq * cp + M.m2 * b * cp * cp + M.m1 * b * pHc;
    }
    curv += kap * cv;
  }
  return curv;
}

// Smallest distance over candidate pairs at x (thread partial; kInf if none).
template <bool LDS>
__device__ __forceinline__ double pairs_dmin(const View& V, const Shared& S, const Tile& T, const double* x,
                                             int& nactive) {
  double dmin = kInf;
  for (int i = threadIdx.x; i < V.npairs; i += blockDim.x) {
    int2 pr = make_int2(0, 0);
    uint64_t rec = 0;
    if constexpr (LDS) rec = V.pslot[i];
    else pr = V.pairs[i];
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    dmin = fmin(dmin, d);
    if (d < V.E->dhat) ++nactive;
  }
  return dmin;
}

// Conservative advancement: largest t <= amax keeping each pair at >= kCcdGap of its
// distance at x, gel points moving along p, indenter static (thread partial min).
// The distance at x comes from the per-pair cache, so pairs that cannot close
// their gap within amax cost only the look-up of p at their gel vertices.
// LDS path: gx = x, gq = p.
template <bool LDS>
__device__ __forceinline__ double pairs_ccd(const View& V, const Shared& S, const Tile& T, const double* x,
                                            const double* p, double amax) {
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  double tmin = amax;
  for (int i = threadIdx.x; i < V.npairs; i += blockDim.x) {
    int2 pr = make_int2(0, 0);
    uint64_t rec = 0;
    if constexpr (LDS) rec = V.pslot[i];
    else pr = V.pairs[i];
    const double d0 = V.pd[i];
    if (!(d0 > 0.0)) { tmin = 0.0; continue; }
    double sk[4] = {0.0, 0.0, 0.0, 0.0};
    int kind;
    if constexpr (LDS) {
      kind = rec_kind(rec);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!point_is_gel(kind, k)) continue;
        const int q = rec_slot(rec, k);
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) s += T.gq[c][q] * T.gq[c][q];
        sk[k] = s;
      }
    } else {
      int id[4];
      pair_point_ids(G, *V.I, pr, id);
      kind = (int)((unsigned)pr.x >> kKindShift);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!point_is_gel(kind, k)) continue;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) { const double pc = p[c * nv + id[k]]; s += pc * pc; }
        sk[k] = s;
      }
    }
    const double l = closing_rate(V.selfc, kind, sk);
    const double gap = kCcdGap * d0;
    if (l * amax <= d0 - gap) continue;
    double t = 0.0, d = d0;
    for (int it = 0; it < kCcdMaxAdvance; ++it) {
      if (l * (amax - t) <= d - gap) { t = amax; break; }
      t += (d - gap) / l;
      PairPts Q;
      get_pair<LDS>(V, S, T, pr, rec, x, p, t, Q);
      if constexpr (LDS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int q = Q.gid[k];
          if (q < 0) continue;
#pragma unroll
          for (int c = 0; c < 3; ++c) Q.z[k][c] = fma(t, T.gq[c][q], Q.z[k][c]);
        }
      }
      Feature g;
      classify(Q, g);
      double r[3];
      d = pair_distance(Q, g, r);
      if (d - gap <= 1e-3 * (d0 - gap)) break;
    }
    tmin = fmin(tmin, fmin(t, amax));
  }
  return tmin;
}

// ---------------------------------------------------------------------------
// Lagged friction (Supp. A, eqs. friction_energy, friction_mollifier)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fric_gslot(const FricPair& F, int k) { return (int)(F.slot >> (10 * k)) & 1023; }
__device__ __forceinline__ int fric_islot(const FricPair& F, int k) { return (int)(F.slot >> (32 + 10 * k)) & 1023; }

// Tangential relative displacement input: Dl = sum a x - sum c y - base.
template <bool LDS>
__device__ __forceinline__ void fric_delta(const View& V, const Shared& S, const Tile& T, const FricPair& F,
                                           const double* x, const double* p, double alpha, double Dl[3]) {
  const int nv = V.G->n_v;
  const IndDev& I = *V.I;
  #pragma unroll
  for (int c = 0; c < 3; ++c) Dl[c] = -F.base[c];
  #pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (F.gv[k] < 0) continue;
    if constexpr (LDS) {
      const int q = fric_gslot(F, k);
      #pragma unroll
      for (int c = 0; c < 3; ++c) Dl[c] += F.a[k] * T.gx[c][q];
    } else {
      const int v = F.gv[k];
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double xv = x[c * nv + v];
        Dl[c] += F.a[k] * (p ? fma(alpha, p[c * nv + v], xv) : xv);
      }
    }
  }
  #pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (F.iv[k] < 0) continue;
    double y[3];
    if constexpr (LDS) {
      const int q = fric_islot(F, k);
      #pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = T.iy[c][q];
    } else {
      ind_world(S, I, F.iv[k], y);
    }
    #pragma unroll
    for (int c = 0; c < 3; ++c) Dl[c] -= F.c[k] * y[c];
  }
}

template <bool LDS>
__device__ __forceinline__ double fric_eval(const View& V, const Shared& S, Tile& T, const double* x,
                                            const double* p, double alpha, double* gout, double* dout) {
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  const double eps = V.E->eps_v;
  double energy = 0.0;
  for (int i = item_first(V); i < V.nfric; i += item_step(V)) {
    const FricPair F = V.fric[i];
    double Dl[3];
    fric_delta<LDS>(V, S, T, F, x, p, alpha, Dl);
    const double nD = dot3(F.n, Dl);
    double TD[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) TD[c] = Dl[c] - nD * F.n[c];
    const double s = sqrt(dot3(TD, TD));
    double f, fos, corr;
    mollifier3(s, eps, f, fos, corr);
    energy += F.mulam * f;
    double uh[3] = {0, 0, 0};
    if (s > 0) for (int c = 0; c < 3; ++c) uh[c] = TD[c] / s;
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int v = F.gv[k];
      if (v < 0) continue;
      if (!LDS && G.fixed[v]) continue;
      const double a = F.a[k];
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double h = fos * (1.0 - F.n[c] * F.n[c]) + corr * uh[c] * uh[c];
        const double gval = F.mulam * a * fos * TD[c], dval = F.mulam * a * a * h;
        if constexpr (LDS) {
          const int q = fric_gslot(F, k);
          atomicAdd(&T.gq[c][q], gval);
          atomicAdd(&T.gd[c][q], dval);
        } else {
          atomicAdd(&gout[c * nv + v], gval);
          atomicAdd(&dout[c * nv + v], dval);
        }
      }
    }
  }
  return energy;
}

template <bool LDS>
__device__ __forceinline__ double fric_curv(const View& V, const Shared& S, const Tile& T, const double* x,
                                            const double* p) {
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  const double eps = V.E->eps_v;
  double curv = 0.0;
  for (int i = threadIdx.x; i < V.nfric; i += blockDim.x) {
    const FricPair F = V.fric[i];
    double Dl[3];
    fric_delta<LDS>(V, S, T, F, x, nullptr, 0.0, Dl);
    const double nD = dot3(F.n, Dl);
    double TD[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) TD[c] = Dl[c] - nD * F.n[c];
    const double s = sqrt(dot3(TD, TD));
    double f, fos, corr;
    mollifier3(s, eps, f, fos, corr);
    double q[3] = {0, 0, 0};
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int v = F.gv[k];
      if (v < 0) continue;
      if constexpr (LDS) {
        const int sl = fric_gslot(F, k);
        #pragma unroll
        for (int c = 0; c < 3; ++c) q[c] += F.a[k] * T.gq[c][sl];
      } else {
        #pragma unroll
        for (int c = 0; c < 3; ++c) q[c] += F.a[k] * p[c * nv + v];
      }
    }
    const double nq = dot3(F.n, q);
    double uq = 0.0;
    if (s > 0) uq = dot3(TD, q) / s;
    curv += F.mulam * (fos * (dot3(q, q) - nq * nq) + corr * uq * uq);
  }
  return curv;
}

// ---------------------------------------------------------------------------
// Broad phase: each gel surface primitive queries a uniform grid of the
// indenter's primitives in the indenter's local frame. A pair is reported from
// the single cell holding the lowest corner of the two boxes' overlap.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_of(double v, double o, double inv, int dim) {
  int c = (int)floor((v - o) * inv);
  return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

// Writes the friction record of a pair closer than dhat at the lag state.
// id: vertex ids of the four points; rec: the pair's slot record (used only
// when the env has slots).
__device__ __forceinline__ void make_fric(const View& V, const PairPts& P, const Feature& f, const double r[3],
                                          double d, const int id[4], uint64_t rec, double muf, FricPair& F) {
  const EnvDev& E = *V.E;
  const int kind = P.kind;
  const double sgn = (kind == kFV) ? -1.0 : 1.0;  // r = gel - indenter for VF and EE
  #pragma unroll
  for (int c = 0; c < 3; ++c) F.n[c] = sgn * r[c] / d;
  #pragma unroll
  for (int k = 0; k < 3; ++k) { F.gv[k] = -1; F.iv[k] = -1; F.a[k] = 0.0; F.c[k] = 0.0; }
  uint64_t gs = 0x3fffffffull, is = 0x3fffffffull;  // three 10-bit kNoSlot10 fields each
  int ng = 0, ni = 0;
  #pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t q = (uint64_t)rec_slot(rec, k) & 1023u;
    if (point_is_gel(kind, k)) {
      F.gv[ng] = id[k];
      F.a[ng] = sgn * f.c[k];
      gs = (gs & ~(1023ull << (10 * ng))) | (q << (10 * ng));
      ++ng;
    } else {
      F.iv[ni] = id[k];
      F.c[ni] = -sgn * f.c[k];
      is = (is & ~(1023ull << (10 * ni))) | (q << (10 * ni));
      ++ni;
    }
  }
  F.slot = gs | (is << 32);
  #pragma unroll
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    #pragma unroll
    for (int k = 0; k < 4; ++k) s += sgn * f.c[k] * P.z[k][c];  // gel cp - indenter cp
    F.base[c] = s;
  }
  double b, b1, b2;
  barrier3(d, E.dhat, b, b1, b2);
  F.mulam = -muf * E.kappa * b1;
}

// Coarse candidates (exact distance < thr) into V.outer, at most cap of them
// (S.overflow set beyond). Returns the thread's smallest distance.
__device__ __forceinline__ double cull(View& V, Shared& S, const double* x, double thr, int cap) {
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const int nv = G.n_v;
  if (threadIdx.x == 0) { S.count = 0; S.overflow = 0; }
  __syncthreads();
  double dmin = kInf;
  const int ntot = G.n_sv + G.n_se + G.n_sf;
  for (int i = item_first(V); i < ntot; i += item_step(V)) {
    int kind, gp, gvid[3], ngv;
    if (i < G.n_sv) { kind = kVF; gvid[0] = G.surf_v[i]; gp = gvid[0]; ngv = 1; }  // VF pairs store the vertex id
    else if (i < G.n_sv + G.n_se) {
      kind = kEE; gp = i - G.n_sv; gvid[0] = G.surf_e[gp]; gvid[1] = G.surf_e[G.n_se + gp]; ngv = 2;
    } else {
      kind = kFV; gp = i - G.n_sv - G.n_se;
      gvid[0] = G.surf_f[gp]; gvid[1] = G.surf_f[G.n_sf + gp]; gvid[2] = G.surf_f[2 * G.n_sf + gp]; ngv = 3;
    }
    double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    for (int k = 0; k < ngv; ++k)
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double xv = x[c * nv + gvid[k]];
        lo[c] = fmin(lo[c], xv);
        hi[c] = fmax(hi[c], xv);
      }
    bool away = false;
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] -= thr; hi[c] += thr;
      if (lo[c] > S.iw_hi[c] || hi[c] < S.iw_lo[c]) away = true;
    }
    if (away) continue;
    // query box in the indenter frame
    double ql[3], qh[3];
    {
      double c[3], h[3];
      #pragma unroll
      for (int k = 0; k < 3; ++k) { c[k] = 0.5 * (lo[k] + hi[k]) - S.t[k]; h[k] = 0.5 * (hi[k] - lo[k]); }
      #pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double cl = S.R[0 * 3 + a] * c[0] + S.R[1 * 3 + a] * c[1] + S.R[2 * 3 + a] * c[2];
        const double hl = fabs(S.R[0 * 3 + a]) * h[0] + fabs(S.R[1 * 3 + a]) * h[1] + fabs(S.R[2 * 3 + a]) * h[2];
        ql[a] = cl - hl;
        qh[a] = cl + hl;
      }
    }
    const Grid& Gr = (kind == kVF) ? I.gf : ((kind == kFV) ? I.gv : I.ge);
    bool outside = false;
    int c0[3], c1[3];
    #pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double gmax = Gr.origin[a] + Gr.dims[a] / Gr.inv_cell;
      if (qh[a] < Gr.origin[a] || ql[a] > gmax) outside = true;
      c0[a] = cell_of(ql[a], Gr.origin[a], Gr.inv_cell, Gr.dims[a]);
      c1[a] = cell_of(qh[a], Gr.origin[a], Gr.inv_cell, Gr.dims[a]);
    }
    if (outside) continue;
    for (int cz = c0[2]; cz <= c1[2]; ++cz)
      for (int cy = c0[1]; cy <= c1[1]; ++cy)
        for (int cx = c0[0]; cx <= c1[0]; ++cx) {
          const int cell = (cz * Gr.dims[1] + cy) * Gr.dims[0] + cx;
          const int j0 = Gr.start[cell], j1 = Gr.start[cell + 1];
          for (int j = j0; j < j1; ++j) {
            const int it = Gr.items[j];
            double il[3], ih[3];
            bool ov = true;
            #pragma unroll
            for (int a = 0; a < 3; ++a) {
              il[a] = Gr.box[a * Gr.n_prim + it];
              ih[a] = Gr.box[(3 + a) * Gr.n_prim + it];
              if (il[a] > qh[a] || ih[a] < ql[a]) ov = false;
            }
            if (!ov) continue;
            // report from the cell of the overlap's lowest corner only
            const int rx = cell_of(fmax(ql[0], il[0]), Gr.origin[0], Gr.inv_cell, Gr.dims[0]);
            const int ry = cell_of(fmax(ql[1], il[1]), Gr.origin[1], Gr.inv_cell, Gr.dims[1]);
            const int rz = cell_of(fmax(ql[2], il[2]), Gr.origin[2], Gr.inv_cell, Gr.dims[2]);
            if (rx != cx || ry != cy || rz != cz) continue;
            int2 pr;
            pr.x = (kind << kKindShift) | gp;
            pr.y = it;
            PairPts P;
            load_pair(V, S, pr, x, nullptr, 0.0, P);
            Feature f;
            classify(P, f);
            double r[3];
            const double d = pair_distance(P, f, r);
            dmin = fmin(dmin, d);
            if (d < thr) {
              const int slot = atomicAdd(&S.count, 1);
              if (slot < cap) V.outer[slot] = pr;
              else S.overflow = 1;
            }
          }
        }
  }
  __syncthreads();
  return dmin;
}

// Self-contact candidates (option): pairs of gel surface primitives sharing no
// vertex (vertex / triangle, edge / edge, each unordered edge pair once) whose
// exact distance is below thr, appended to V.outer after the indenter pairs.
// Searched among the surface primitives all of whose vertices are gel points of
// the coarse list, i.e. within its margin of the indenter, where the gel
// deforms, by pairwise box tests. The region's vertex, triangle and edge lists
// are staged in the inner list's storage (rebuilt by the refilter that follows
// every coarse build); a region beyond that storage sets S.overflow.
__device__ __forceinline__ void cull_self(View& V, Shared& S, const double* x, double thr, int cap, int pair_cap) {
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const int nv = G.n_v;
  const int n0 = min(S.count, cap);
  for (int i = threadIdx.x; i < n0; i += blockDim.x) {
    const int2 pr = V.outer[i];
    const int kind = (int)((unsigned)pr.x >> kKindShift);
    int id[4];
    pair_point_ids(G, I, pr, id);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (point_is_gel(kind, k)) V.vmap[id[k]] = -1;
  }
  if (threadIdx.x == 0) { S.rcount[0] = 0; S.rcount[1] = 0; S.rcount[2] = 0; }
  __syncthreads();
  T2R_G int* rv = reinterpret_cast<T2R_G int*>(V.pairs);  // 2 pair_cap ints
  const int cap_v = min(kGelSlots, pair_cap / 2), cap_fe = (2 * pair_cap - cap_v) / 2;
  T2R_G int* rf = rv + cap_v;
  T2R_G int* re = rf + cap_fe;
  for (int i = item_first(V); i < G.n_sv; i += item_step(V)) {
    const int v = G.surf_v[i];
    if (V.vmap[v] != -1) continue;
    const int q = atomicAdd(&S.rcount[0], 1);
    if (q < cap_v) rv[q] = v;
    else S.overflow = 1;
  }
  for (int i = item_first(V); i < G.n_sf; i += item_step(V)) {
    if (V.vmap[G.surf_f[i]] != -1 || V.vmap[G.surf_f[G.n_sf + i]] != -1 || V.vmap[G.surf_f[2 * G.n_sf + i]] != -1)
      continue;
    const int q = atomicAdd(&S.rcount[1], 1);
    if (q < cap_fe) rf[q] = i;
    else S.overflow = 1;
  }
  for (int i = item_first(V); i < G.n_se; i += item_step(V)) {
    if (V.vmap[G.surf_e[i]] != -1 || V.vmap[G.surf_e[G.n_se + i]] != -1) continue;
    const int q = atomicAdd(&S.rcount[2], 1);
    if (q < cap_fe) re[q] = i;
    else S.overflow = 1;
  }
  __syncthreads();
  const int nrv = min(S.rcount[0], cap_v), nrf = min(S.rcount[1], cap_fe), nre = min(S.rcount[2], cap_fe);
  auto near = [&](const double lo[3], const double hi[3], const double lo2[3], const double hi2[3]) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) ok = ok && lo[c] - thr <= hi2[c] && lo2[c] - thr <= hi[c];
    return ok;
  };
  auto append = [&](int kind, int a, int b) {
    int2 pr;
    pr.x = (kind << kKindShift) | a;
    pr.y = b;
    PairPts P;
    load_pair(V, S, pr, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    if (!(pair_distance(P, f, r) < thr)) return;
    const int slot = atomicAdd(&S.count, 1);
    if (slot < cap) V.outer[slot] = pr;
    else S.overflow = 1;
  };
  const long long nvf = (long long)nrv * nrf;
  for (long long k = item_first(V); k < nvf; k += item_step(V)) {
    const int v = rv[k / nrf], f = rf[k % nrf];
    const int t3[3] = {G.surf_f[f], G.surf_f[G.n_sf + f], G.surf_f[2 * G.n_sf + f]};
    if (v == t3[0] || v == t3[1] || v == t3[2]) continue;
    double lo[3], hi[3], pv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv[c] = x[c * nv + v];
      lo[c] = fmin(fmin(x[c * nv + t3[0]], x[c * nv + t3[1]]), x[c * nv + t3[2]]);
      hi[c] = fmax(fmax(x[c * nv + t3[0]], x[c * nv + t3[1]]), x[c * nv + t3[2]]);
    }
    if (near(pv, pv, lo, hi)) append(kGVF, v, f);
  }
  const long long nee = (long long)nre * nre;
  for (long long k = item_first(V); k < nee; k += item_step(V)) {
    const int ia = (int)(k / nre), ib = (int)(k % nre);
    if (ia >= ib) continue;
    const int ea = re[ia], eb = re[ib];
    const int a0 = G.surf_e[ea], a1 = G.surf_e[G.n_se + ea], b0 = G.surf_e[eb], b1 = G.surf_e[G.n_se + eb];
    if (a0 == b0 || a0 == b1 || a1 == b0 || a1 == b1) continue;
    double lo[3], hi[3], lo2[3], hi2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(x[c * nv + a0], x[c * nv + a1]);
      hi[c] = fmax(x[c * nv + a0], x[c * nv + a1]);
      lo2[c] = fmin(x[c * nv + b0], x[c * nv + b1]);
      hi2[c] = fmax(x[c * nv + b0], x[c * nv + b1]);
    }
    if (near(lo, hi, lo2, hi2)) append(kGEE, ea, eb);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Vector passes over the 3 n_v DOFs of an env
// ---------------------------------------------------------------------------
struct Solver {
  View V;
  Shared* S;
  Tile* T;
  double floor_d;     // preconditioner floor
  double guard;       // energy rounding guard
  double buffer;      // inner list radius beyond dhat
  double buffer_out;  // outer list radius beyond dhat
  int armijo;
  int pair_cap, fric_cap, outer_cap;
  ListState* L;       // persistent list state of this env
  double* xs_o;       // [3][n_sv] surface positions at the outer build
  double* xs_i;       // [3][n_sv] ... at the inner build
  // stats
  int reculls, restarts, halvings, ncand, outer_builds;
  double fill;        // largest list length / capacity seen
  // work budget: energy and curvature evaluation passes of this env in this launch
  long long evals, max_evals;
  int mixed0;         // configured precision (a solve's line-search fallback may switch to FP64)
  int fallbacks;      // line-search fallbacks taken in the current solve
};

// Inner candidate list from the outer one: exact distance of every coarse pair,
// keep those below thr. Work is one pair per thread, so it stays balanced.
template <bool LDS>
__device__ __forceinline__ void filter_pairs(View& V, Shared& S, const Tile& T, const double* x, double thr,
                                             int cap) {
  if (threadIdx.x == 0) { S.count = 0; S.overflow = 0; }
  __syncthreads();
  for (int i = item_first(V); i < V.nouter; i += item_step(V)) {
    const int2 pr = V.outer[i];
    const uint64_t rec = LDS ? V.oslot[i] : 0ull;
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    if (d < thr) {
      const int slot = atomicAdd(&S.count, 1);
      if (slot < cap) {
        V.pairs[slot] = pr;
        V.pd[slot] = d;
        V.pslot[slot] = rec;
      } else {
        S.overflow = 1;
      }
    }
  }
  __syncthreads();
}

// Largest displacement of any indenter point between two poses:
// |dt| + 2 sin(theta/2) r_max, theta the relative rotation angle; sin(theta/2)
// is the norm of the vector part of q_b conj(q_a) (unit quaternions), which
// stays accurate for small angles.
__device__ __forceinline__ double ind_motion(const double a[7], const double b[7], double r_max) {
  double dt = 0.0, na = 0.0, nb = 0.0;
  for (int i = 0; i < 3; ++i) dt += (a[i] - b[i]) * (a[i] - b[i]);
  for (int i = 3; i < 7; ++i) { na += a[i] * a[i]; nb += b[i] * b[i]; }
  const double wa = a[3], wb = b[3];
  const double va[3] = {a[4], a[5], a[6]}, vb[3] = {b[4], b[5], b[6]};
  double v[3];
  v[0] = wa * vb[0] - wb * va[0] - (vb[1] * va[2] - vb[2] * va[1]);
  v[1] = wa * vb[1] - wb * va[1] - (vb[2] * va[0] - vb[0] * va[2]);
  v[2] = wa * vb[2] - wb * va[2] - (vb[0] * va[1] - vb[1] * va[0]);
  const double sh = fmin(1.0, sqrt((v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (na * nb)));
  return sqrt(dt) + 2.0 * sh * r_max * (1.0 + 1e-12);
}

// Largest surface-vertex displacement since each snapshot and largest |p| on the
// surface (p may be null): out = {outer, inner, p}.
// Motion of the gel surface relative to the indenter since each list was built
// (out[0]: outer list, out[1]: inner list) and max |p| over the surface
// (out[2]). A surface vertex's relative motion is its distance from its
// snapshot position carried along with the indenter's rigid motion since the
// build, M (g - t_b) + t (M = R R_b^T). For a gel point g and an indenter
// point y at distance D at the build, their distance changes by at most that
// motion (a convex combination over the primitive's vertices) plus
// |(M - I)(y - g)| <= theta D, theta the rotation angle since the build; a
// pair beyond the list radius r then stays beyond r - (motion + theta r), so
// theta r is added to each list's figure.
__device__ __forceinline__ void surf_motion(Solver& s, const double* x, const double* p, double out[5]) {
  const GelDev& G = *s.V.G;
  const int nv = G.n_v, ns = G.n_sv;
  const Shared& S = *s.S;
  double Mo[9], Mi[9], to[3], ti[3];
  double th[2];
  {
    const double* pb[2] = {s.L->pose_o, s.L->pose_i};
    double* Mx[2] = {Mo, Mi};
    double* tx[2] = {to, ti};
    for (int l = 0; l < 2; ++l) {
      double Rb[9];
      quat_to_R(pb[l] + 3, Rb);
      #pragma unroll
      for (int r = 0; r < 3; ++r)
        #pragma unroll
        for (int c = 0; c < 3; ++c)
          Mx[l][r * 3 + c] = S.R[r * 3 + 0] * Rb[c * 3 + 0] + S.R[r * 3 + 1] * Rb[c * 3 + 1] +
                             S.R[r * 3 + 2] * Rb[c * 3 + 2];
      #pragma unroll
      for (int c = 0; c < 3; ++c) tx[l][c] = pb[l][c];
      double qa = 0.0, na = 0.0, nb = 0.0;
      for (int i = 3; i < 7; ++i) { qa += pb[l][i] * S.pose[i]; na += pb[l][i] * pb[l][i]; nb += S.pose[i] * S.pose[i]; }
      th[l] = 2.0 * acos(fmin(1.0, fabs(qa) / sqrt(na * nb)));
    }
  }
  double m[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const int v = G.surf_v[i];
    double go[3], gi[3], xv[3];
    double c2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xv[c] = x[c * nv + v];
      go[c] = s.xs_o[c * ns + i] - to[c];
      gi[c] = s.xs_i[c * ns + i] - ti[c];
      if (p) { const double pv = p[c * nv + v]; c2 += pv * pv; }
    }
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double da = xv[r] - (Mo[r * 3 + 0] * go[0] + Mo[r * 3 + 1] * go[1] + Mo[r * 3 + 2] * go[2] + S.t[r]);
      const double db = xv[r] - (Mi[r * 3 + 0] * gi[0] + Mi[r * 3 + 1] * gi[1] + Mi[r * 3 + 2] * gi[2] + S.t[r]);
      a += da * da;
      b += db * db;
    }
    m[0] = fmax(m[0], a);
    m[1] = fmax(m[1], b);
    m[2] = fmax(m[2], c2);
  }
  block_reduce<0, 3>(m, *s.S);
  const double dh = s.V.E->dhat;
  out[0] = sqrt(m[0]) + th[0] * (dh + s.buffer_out);
  out[1] = sqrt(m[1]) + th[1] * (dh + s.buffer);
  out[2] = sqrt(m[2]);
  // deviation from the indenter's rigid motion alone: the distance of two gel
  // points changes by at most twice it (a rigid motion keeps their distance)
  out[3] = sqrt(m[0]);
  out[4] = sqrt(m[1]);
}

__device__ __forceinline__ void snapshot(Solver& s, const double* x, double* dst) {
  const GelDev& G = *s.V.G;
  const int nv = G.n_v, ns = G.n_sv;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const int v = G.surf_v[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c * ns + i] = x[c * nv + v];
  }
  __syncthreads();
}

// Contact slots of the outer list: every gel and indenter vertex of an outer
// pair or a friction pair gets a dense slot (slot_v / islot_v map back), each
// outer pair gets its record (slots of its four points and its kind) and each
// friction pair its slots. More than kGelSlots gel or kIndSlots indenter
// vertices: slots_ok = 0 and the pair passes use the global path. The maps
// vmap / imap are all zero again on return.
__device__ __forceinline__ void build_slots(Solver& s) {
  View& V = s.V;
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  Shared& S = *s.S;
  for (int i = threadIdx.x; i < V.nouter; i += blockDim.x) {
    const int2 pr = V.outer[i];
    const int kind = (int)((unsigned)pr.x >> kKindShift);
    int id[4];
    pair_point_ids(G, I, pr, id);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (point_is_gel(kind, k)) V.vmap[id[k]] = -1;
      else V.imap[id[k]] = -1;
    }
  }
  for (int i = threadIdx.x; i < V.nfric; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (V.fric[i].gv[k] >= 0) V.vmap[V.fric[i].gv[k]] = -1;
      if (V.fric[i].iv[k] >= 0) V.imap[V.fric[i].iv[k]] = -1;
    }
  }
  if (threadIdx.x == 0) { S.count = 0; S.overflow = 0; }
  __syncthreads();
  for (int v = threadIdx.x; v < G.n_v; v += blockDim.x) {
    if (V.vmap[v] == -1) {
      const int q = atomicAdd(&S.count, 1);
      if (q < kGelSlots) { V.vmap[v] = q + 1; V.slot_v[q] = v; }
    }
  }
  for (int j = threadIdx.x; j < I.n_v; j += blockDim.x) {
    if (V.imap[j] == -1) {
      const int q = atomicAdd(&S.overflow, 1);
      if (q < kIndSlots) { V.imap[j] = q + 1; V.islot_v[q] = j; }
    }
  }
  __syncthreads();
  const int ng = S.count, ni = S.overflow;
  const int ok = ng <= kGelSlots && ni <= kIndSlots;
  if (ok) {
    for (int i = threadIdx.x; i < V.nouter; i += blockDim.x) {
      const int2 pr = V.outer[i];
      const int kind = (int)((unsigned)pr.x >> kKindShift);
      int id[4];
      pair_point_ids(G, I, pr, id);
      uint64_t rec = (uint64_t)kind << (4 * kRecBits);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int m = point_is_gel(kind, k) ? V.vmap[id[k]] : V.imap[id[k]];
        rec |= (uint64_t)(m - 1) << (kRecBits * k);
      }
      V.oslot[i] = rec;
    }
    for (int i = threadIdx.x; i < V.nfric; i += blockDim.x) {
      uint64_t gs = 0, is = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int gv = V.fric[i].gv[k], iv = V.fric[i].iv[k];
        gs |= (uint64_t)(gv >= 0 ? V.vmap[gv] - 1 : (int)kNoSlot10) << (10 * k);
        is |= (uint64_t)(iv >= 0 ? V.imap[iv] - 1 : (int)kNoSlot10) << (10 * k);
      }
      V.fric[i].slot = gs | (is << 32);
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < G.n_v; v += blockDim.x) V.vmap[v] = 0;
  for (int j = threadIdx.x; j < I.n_v; j += blockDim.x) V.imap[j] = 0;
  V.slots_ok = ok;
  V.nslots = ok ? ng : 0;
  V.nislots = ok ? ni : 0;
  if (threadIdx.x == 0) {
    s.L->slots_ok = ok;
    s.L->n_slots = V.nslots;
    s.L->n_islots = V.nislots;
  }
  __syncthreads();
}

// Two-level neighbour list. The outer list (radius dhat + buffer_out) comes from
// the grid traversal; the inner list (radius dhat + buffer) filters it. Each
// list remembers the surface positions and the indenter pose it was built at.
// A pair's distance changes by at most the motion of its gel points plus that of
// the indenter, so a pair missing from the inner list is still inactive and
// cannot be hit as long as (surface motion + indenter motion + the coming step)
// stays below buffer; for the outer list the margin is buffer_out - buffer,
// which also keeps every pair within the inner radius inside the outer list.
__device__ __forceinline__ bool rebuild_outer(Solver& s, const double* x) {
  View& V = s.V;
  const unsigned long long t0 = tick();
  cull(V, *s.S, x, V.E->dhat + s.buffer_out, s.outer_cap);
  if (V.selfc) cull_self(V, *s.S, x, V.E->dhat + s.buffer_out, s.outer_cap, s.pair_cap);
  const int ov = s.S->overflow;
  const int cnt = s.S->count;
  __syncthreads();
  V.nouter = min(cnt, s.outer_cap);
  s.fill = fmax(s.fill, (double)cnt / s.outer_cap);
  snapshot(s, x, s.xs_o);
  build_slots(s);
  if (threadIdx.x == 0) {
    for (int i = 0; i < 7; ++i) s.L->pose_o[i] = s.S->pose[i];
    s.L->n_outer = V.nouter;
    s.L->valid_o = ov ? 0 : 1;
    s.L->valid_i = 0;
  }
  ++s.outer_builds;
  __syncthreads();
  tock(*s.S, 0, t0);
  return ov == 0;
}

__device__ __forceinline__ bool refilter(Solver& s, const double* x) {
  View& V = s.V;
  const unsigned long long t0 = tick();
  if (V.slots_ok) {
    stage_points(V, *s.S, *s.T, x, nullptr, 0.0, 0);
    filter_pairs<true>(V, *s.S, *s.T, x, V.E->dhat + s.buffer, s.pair_cap);
  } else {
    filter_pairs<false>(V, *s.S, *s.T, x, V.E->dhat + s.buffer, s.pair_cap);
  }
  const int ov = s.S->overflow;
  const int cnt = s.S->count;
  __syncthreads();
  V.npairs = min(cnt, s.pair_cap);
  s.fill = fmax(s.fill, (double)cnt / s.pair_cap);
  s.ncand = V.npairs;
  ++s.reculls;
  snapshot(s, x, s.xs_i);
  if (threadIdx.x == 0) {
    for (int i = 0; i < 7; ++i) s.L->pose_i[i] = s.S->pose[i];
    s.L->n_inner = V.npairs;
    s.L->valid_i = ov ? 0 : 1;
  }
  __syncthreads();
  tock(*s.S, 1, t0);
  return ov == 0;
}

// Makes both lists valid at (x, current pose) for a coming motion of at most
// `step` of any surface point. Returns false on a list overflow.
__device__ __forceinline__ bool ensure_lists(Solver& s, const double* x, double step, const double m[5]) {
  const int vo = s.L->valid_o, vi = s.L->valid_i;
  double mo = vo ? m[0] : kInf;  // relative motions since the builds (surf_motion)
  double mi = vi ? m[1] : kInf;
  if (s.V.selfc) {  // gel-gel pairs: both points move, up to the deviation and the step each
    mo = fmax(mo, vo ? 2.0 * m[3] + step : kInf);
    mi = fmax(mi, vi ? 2.0 * m[4] + step : kInf);
  }
  __syncthreads();
  if (!(mo + step <= s.buffer_out - s.buffer)) {
    if (!rebuild_outer(s, x)) return false;
    return refilter(s, x);
  }
  if (!(mi + step <= s.buffer)) return refilter(s, x);
  return true;
}

__device__ __forceinline__ bool ensure_lists(Solver& s, const double* x, double step) {
  double m[5];
  surf_motion(s, x, nullptr, m);
  return ensure_lists(s, x, step, m);
}

// Restores the list sizes kept from the previous launch.
__device__ __forceinline__ void load_lists(Solver& s) {
  s.V.nouter = s.L->valid_o ? s.L->n_outer : 0;
  s.V.npairs = s.L->valid_i ? s.L->n_inner : 0;
  s.V.slots_ok = s.L->valid_o ? s.L->slots_ok : 0;
  s.V.nslots = s.V.slots_ok ? s.L->n_slots : 0;
  s.V.nislots = s.V.slots_ok ? s.L->n_islots : 0;
}

// Friction lag and smallest distance at (x, current pose) from the outer list:
// exact distance of every coarse pair; pairs closer than dhat get a friction
// record when mode == 1. Requires a valid outer list. Returns the thread's min d.
template <bool LDS>
__device__ __forceinline__ double lag_pass(Solver& s, const double* x, int mode, double muf) {
  View& V = s.V;
  Shared& S = *s.S;
  const Tile& T = *s.T;
  if (threadIdx.x == 0) { S.count = 0; S.overflow = 0; }
  __syncthreads();
  double dmin = kInf;
  for (int i = item_first(V); i < V.nouter; i += item_step(V)) {
    const int2 pr = V.outer[i];
    const uint64_t rec = LDS ? V.oslot[i] : 0ull;
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    dmin = fmin(dmin, d);
    if (mode == 1 && P.kind < kGVF && d < V.E->dhat && d > 0.0) {  // self-contact pairs: no friction
      const int slot = atomicAdd(&S.count, 1);
      if (slot < s.fric_cap) {
        int id[4];
        pair_point_ids(*V.G, *V.I, pr, id);
        make_fric(V, P, f, r, d, id, rec, muf, V.fric[slot]);
      } else {
        S.overflow = 1;
      }
    }
  }
  __syncthreads();
  return dmin;
}

// muf: the friction coefficient the records carry (the env's own, or 1 for the
// derivative with respect to it).
__device__ __forceinline__ double lag_from_outer(Solver& s, const double* x, int mode, double muf) {
  if (s.V.slots_ok) {
    stage_points(s.V, *s.S, *s.T, x, nullptr, 0.0, 0);
    return lag_pass<true>(s, x, mode, muf);
  }
  return lag_pass<false>(s, x, mode, muf);
}

// Smallest pair distance and active count at x over the inner list (block-wide).
__device__ __forceinline__ double dmin_all(Solver& s, const double* x, int& nactive) {
  View& V = s.V;
  int na = 0;
  double dm;
  if (V.slots_ok) {
    stage_points(V, *s.S, *s.T, x, nullptr, 0.0, 0);
    dm = pairs_dmin<true>(V, *s.S, *s.T, x, na);
  } else {
    dm = pairs_dmin<false>(V, *s.S, *s.T, x, na);
  }
  double w[2] = {(double)na, -dm};
  block_reduce<1, 1>(w, *s.S);
  nactive = (int)w[0];
  return -w[1];
}

// Evaluates Pi, grad (-> g) and diag at x + alpha p. Returns energy; feasible in flag.
// Inertia term of the dynamic form (Supp. A, eq. ipc_energy): at x + alpha p,
// 1/2 w_v |x_v - xhat_v|^2 with w_v = m_v / dt^2 and xhat = x^t + dt v^t
// (x^t = xprev during a load step); its gradient and diagonal are added to
// g and dg (free DOFs; every earlier pass's sums are in place). Returns the
// thread's energy partial.
__device__ __forceinline__ double inertia_eval(const View& V, const Shared& S, const double* x, const double* p,
                                               double alpha, double* g, double* dg) {
  const GelDev& G = *V.G;
  const int nv = G.n_v, n = 3 * nv;
  double e = 0.0;
  __syncthreads();
  const int B = blockDim.x;
  const double* vel = S.vel;
  // two entries per thread and trip, every load first (same per-thread order; eight
  // values per entry, so four would hold too many registers)
  constexpr int U = 2;
  for (int j0 = threadIdx.x; j0 < n; j0 += U * B) {
    bool fx[U];
    double mv[U], xv[U], pv[U], vv[U], qv[U], gv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = min(j0 + u * B, n - 1);  // clamped: the loads issue unconditionally
      const int v = j >= 2 * nv ? j - 2 * nv : (j >= nv ? j - nv : j);
      fx[u] = G.fixed[v];
      mv[u] = G.vmass[v];
      xv[u] = x[j];
      pv[u] = p ? p[j] : 0.0;
      vv[u] = vel[j];
      qv[u] = V.xprev[j];
      gv[u] = g[j];
      dv[u] = dg[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * B;
      if (j >= n || fx[u]) continue;
      const double w = S.iw * mv[u];
      const double xt = p ? fma(alpha, pv[u], xv[u]) : xv[u];
      const double r = xt - fma(S.dt, vv[u], qv[u]);
      g[j] = gv[u] + w * r;
      dg[j] = dv[u] + w;
      e += 0.5 * w * r * r;
    }
  }
  return e;
}

// p^T (inertia Hessian) p: sum over free DOFs of w_v p^2 (thread partial).
__device__ __forceinline__ double inertia_curv(const View& V, const Shared& S, const double* p) {
  const GelDev& G = *V.G;
  const int nv = G.n_v, n = 3 * nv;
  double c = 0.0;
  const int B = blockDim.x;
  for (int j0 = threadIdx.x; j0 < n; j0 += kVecUnroll * B) {
    bool fx[kVecUnroll];
    double mv[kVecUnroll], pv[kVecUnroll];
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const int j = min(j0 + u * B, n - 1);
      const int v = j >= 2 * nv ? j - 2 * nv : (j >= nv ? j - nv : j);
      fx[u] = G.fixed[v];
      mv[u] = G.vmass[v];
      pv[u] = p[j];
    }
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u)
      if (j0 + u * B < n && !fx[u]) c += S.iw * mv[u] * pv[u] * pv[u];
  }
  return c;
}

// INERTIA = false leaves the dynamic form's term out of the code (kernels that
// evaluate the quasi-static energy only).
template <bool INERTIA = true>
__device__ __forceinline__ double eval_all(Solver& s, const double* x, const double* p, double alpha, double* g,
                           double* dg, int& feasible, int& nactive, double* e_el = nullptr) {
  View& V = s.V;
  int feas = 1, nact = 0;
  double v[3];
  ++s.evals;
  unsigned long long t0 = tick();
  v[0] = elem_eval(V, x, p, alpha, g, dg, *s.T, feas);
  tock(*s.S, 5, t0);
  double eel = v[0];
  t0 = tick();
  Tile& T = *s.T;
  const Shared& S = *s.S;
  if (V.slots_ok) {
    stage_points(V, S, T, x, p, alpha, 2);
    v[0] += pairs_eval<true>(V, S, T, x, p, alpha, g, dg, feas, nact);
    if (V.nfric > 0) v[0] += fric_eval<true>(V, S, T, x, p, alpha, g, dg);
    flush_slots(V, T, g, dg);
  } else {
    v[0] += pairs_eval<false>(V, S, T, x, p, alpha, g, dg, feas, nact);
    if (V.nfric > 0) v[0] += fric_eval<false>(V, S, T, x, p, alpha, g, dg);
  }
  if constexpr (INERTIA)
    if (S.iw > 0.0) v[0] += inertia_eval(V, S, x, p, alpha, g, dg);
  v[1] = (double)nact;
  v[2] = feas ? 0.0 : 1.0;  // max -> any infeasible
  double w[4] = {v[0], v[1], eel, v[2]};
  block_reduce<3, 1>(w, *s.S);
  tock(*s.S, 6, t0);
  feasible = (w[3] == 0.0);
  nactive = (int)w[1];
  if (e_el) *e_el = w[2];
  return w[0];
}

__device__ __forceinline__ double curvature_all(Solver& s, const double* x, const double* p) {
  View& V = s.V;
  ++s.evals;
  unsigned long long t0 = tick();
  double c = elem_curv(V, x, p, *s.T);
  tock(*s.S, 2, t0);
  t0 = tick();
  Tile& T = *s.T;
  const Shared& S = *s.S;
  if (V.slots_ok) {
    stage_points(V, S, T, x, p, 0.0, 1);
    c += pairs_curv<true>(V, S, T, x, p);
    if (V.nfric > 0) c += fric_curv<true>(V, S, T, x, p);
  } else {
    c += pairs_curv<false>(V, S, T, x, p);
    if (V.nfric > 0) c += fric_curv<false>(V, S, T, x, p);
  }
  if (S.iw > 0.0) c += inertia_curv(V, S, p);
  double w[1] = {c};
  block_reduce<1, 0>(w, *s.S);
  tock(*s.S, 3, t0);
  return w[0];
}

// P = 1/max(diag, floor) stored in place; p = -P g; returns |Pg|_inf, |p|_inf, g.p
__device__ __forceinline__ void init_direction(Solver& s, const double* g, double& res, double& pinf, double& gp) {
  View& V = s.V;
  const int n = 3 * V.G->n_v;
  double a[3] = {0.0, 0.0, 0.0};  // sum g.p ; max |Pg| ; (pinf = res)
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double P = 1.0 / fmax(V.diag[j], s.floor_d);
    V.diag[j] = P;
    const double pj = -P * g[j];
    V.p[j] = pj;
    a[0] += g[j] * pj;
    a[1] = fmax(a[1], fabs(pj));
  }
  double w[2] = {a[0], a[1]};
  block_reduce<1, 1>(w, *s.S);
  gp = w[0];
  res = w[1];
  pinf = w[1];
}

// Runs PNCG at the current pose from x. Returns status bits (kConverged etc.).
__device__ __forceinline__ int pncg(Solver& s, double tol, int max_iters, int& iters, double& res_out, double& e_out,
                    int& nactive_out) {
  View& V = s.V;
  const int n = 3 * V.G->n_v;
  const double dh = V.E->dhat;
  double* x = V.x;
  double* g0 = V.g0;
  double* g1 = V.g1;
  if (s.evals >= s.max_evals) { iters = 0; return kMaxIter | kBudget; }
  V.mixed = s.mixed0;
  s.fallbacks = 0;
  if (!ensure_lists(s, x, 0.0)) return kOverflow;
  int feas, nact;
  unsigned long long t0;
  double E0 = eval_all(s, x, V.p, 0.0, g0, V.diag, feas, nact);
  nactive_out = nact;
  if (!feas) { iters = 0; return kInfeasible; }
  double res, pinf, gp;
  t0 = tick();
  init_direction(s, g0, res, pinf, gp);
  tock(*s.S, 7, t0);
  int status = 0;
  int k = 0;
  for (;; ++k) {
    if (res <= tol) { status = kConverged; break; }
    if (k >= max_iters) { status = kMaxIter; break; }
    if (s.evals >= s.max_evals) { status = kMaxIter | kBudget; break; }
    const double a_up = dh / (2.0 * pinf);
    const double curv = curvature_all(s, x, V.p);
    const double a_bar = (curv > 0.0) ? -gp / curv : kInf;
    double alpha = fmin(a_up, a_bar);
    {
      double m[5];
      surf_motion(s, x, V.p, m);
      if (!ensure_lists(s, x, alpha * m[2], m)) { status = kOverflow; break; }
    }
    t0 = tick();
    {
      double w;
      if (V.slots_ok) {
        stage_points(V, *s.S, *s.T, x, V.p, 0.0, 1);
        w = pairs_ccd<true>(V, *s.S, *s.T, x, V.p, alpha);
      } else {
        w = pairs_ccd<false>(V, *s.S, *s.T, x, V.p, alpha);
      }
      alpha = block_min(w, *s.S);
    }
    tock(*s.S, 4, t0);
    bool ok = false;
    double E1 = E0;
    // rounding guard: the energy sum's rounding noise grows with |Pi| (barrier
    // terms of close pairs dominate it in contact), on top of the elastic scale
    const double guard = s.guard + kEnergyGuard * fabs(E0);
    for (int h = 0; h <= kMaxHalvings; ++h) {
      E1 = eval_all(s, x, V.p, alpha, g1, V.diag, feas, nact);
      if (feas && (!s.armijo || E1 <= E0 + kArmijoC * alpha * gp + guard)) { ok = true; break; }
      alpha *= 0.5;
      ++s.halvings;
    }
    t0 = tick();
    if (!ok) {
      // one fallback per solve: restart along -P g at x; in mixed precision with
      // FP64 element terms for the rest of the solve (FP32 rounding of the
      // element gradient can leave no descent the FP64 energy test accepts)
      if (s.fallbacks > 0) { status = kLineSearch; break; }
      ++s.fallbacks;
      V.mixed = 0;
      E0 = eval_all(s, x, V.p, 0.0, g0, V.diag, feas, nact);
      init_direction(s, g0, res, pinf, gp);
      ++s.restarts;
      tock(*s.S, 7, t0);
      continue;
    }
    nactive_out = nact;
    // dots: x += alpha p ; P1 ; y = g1 - g0
    double a[6] = {0, 0, 0, 0, 0, 0};  // gPy, yPy, yp, pg1, gPg | max|Pg1|
    // kVecUnroll entries per thread per trip, all loads issued first (more bytes in
    // flight per wave); each thread still visits j, j + B, j + 2B, ... in order, so
    // its partial sums are the same as with one entry per trip
    const int B = blockDim.x;
    for (int j0 = threadIdx.x; j0 < n; j0 += kVecUnroll * B) {
      double pv[kVecUnroll], xv[kVecUnroll], dv[kVecUnroll], g1v[kVecUnroll], g0v[kVecUnroll];
#pragma unroll
      for (int u = 0; u < kVecUnroll; ++u) {
        const int j = min(j0 + u * B, n - 1);  // clamped: the loads issue unconditionally
        pv[u] = V.p[j];
        xv[u] = x[j];
        dv[u] = V.diag[j];
        g1v[u] = g1[j];
        g0v[u] = g0[j];
      }
#pragma unroll
      for (int u = 0; u < kVecUnroll; ++u) {
        const int j = j0 + u * B;
        if (j < n) {
          const double pj = pv[u];
          x[j] = fma(alpha, pj, xv[u]);
          const double P = 1.0 / fmax(dv[u], s.floor_d);
          V.diag[j] = P;
          const double gj = g1v[u];
          const double y = gj - g0v[u];
          const double Py = P * y;
          a[0] += gj * Py;
          a[1] += y * Py;
          a[2] += y * pj;
          a[3] += pj * gj;
          a[4] += gj * P * gj;
          a[5] = fmax(a[5], fabs(P * gj));
        }
      }
    }
    block_reduce<5, 1>(a, *s.S);
    const double yp = a[2];
    double beta = 0.0;
    if (yp > kYpMin) beta = a[0] / yp - (a[1] / yp) * (a[3] / yp);
    double b2[2] = {0.0, 0.0};  // g.p_new | max |p_new|
    for (int j0 = threadIdx.x; j0 < n; j0 += kVecUnroll * B) {
      double dv[kVecUnroll], gv[kVecUnroll], pv[kVecUnroll];
#pragma unroll
      for (int u = 0; u < kVecUnroll; ++u) {
        const int j = min(j0 + u * B, n - 1);
        dv[u] = V.diag[j];
        gv[u] = g1[j];
        pv[u] = V.p[j];
      }
#pragma unroll
      for (int u = 0; u < kVecUnroll; ++u) {
        const int j = j0 + u * B;
        if (j < n) {
          const double pn = -dv[u] * gv[u] + beta * pv[u];
          V.p[j] = pn;
          b2[0] += gv[u] * pn;
          b2[1] = fmax(b2[1], fabs(pn));
        }
      }
    }
    block_reduce<1, 1>(b2, *s.S);
    gp = b2[0];
    pinf = b2[1];
    res = a[5];
    if (gp >= 0.0) {  // not a descent direction: restart with -P g
      for (int j = threadIdx.x; j < n; j += blockDim.x) V.p[j] = -V.diag[j] * g1[j];
      __syncthreads();
      gp = -a[4];
      pinf = a[5];
      ++s.restarts;
    }
    E0 = E1;
    double* tmp = g0; g0 = g1; g1 = tmp;
    tock(*s.S, 7, t0);
  }
  iters = k;
  res_out = res;
  e_out = E0;
  // keep the latest gradient in V.g0 for callers
  if (g0 != V.g0) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) V.g0[j] = g0[j];
    __syncthreads();
  }
  return status;
}

__device__ __forceinline__ void make_view(const StepParams& P, int e, View& V) {
  V.E = P.envs + e;
  const EnvDev& E = *V.E;
  V.G = P.gels + E.gel;
  V.I = P.inds + E.ind;
  V.x = P.x + E.voff;
  V.xprev = P.xprev + E.voff;
  V.g0 = P.g0 + E.voff;
  V.g1 = P.g1 + E.voff;
  V.diag = P.diag + E.voff;
  V.p = P.p + E.voff;
  V.pairs = P.pairs + E.poff;
  V.pd = P.pair_d + E.poff;
  V.outer = P.outer + E.ooff;
  V.nouter = 0;
  V.fric = P.fric + E.foff;
  V.vmap = P.vmap + E.vtxoff;
  V.oslot = P.oslot + E.ooff;
  V.pslot = P.pslot + E.poff;
  V.slot_v = P.slot_v + (long long)e * kGelSlots;
  V.imap = P.imap + E.imoff;
  V.islot_v = P.islot_v + (long long)e * kIndSlots;
  V.npairs = 0;
  V.nfric = 0;
  V.nslots = 0;
  V.nislots = 0;
  V.slots_ok = 0;
  V.mixed = P.precision;
  V.moll = P.ee_moll;
  V.det = P.det;
  V.selfc = P.selfc;
}

__device__ __forceinline__ void init_solver(Solver& s, const StepParams& P, Shared& S, Tile& T) {
  const EnvDev& E = *s.V.E;
  const GelDev& G = *s.V.G;
  s.S = &S;
  s.T = &T;
  s.mixed0 = s.V.mixed;
  s.fallbacks = 0;
  s.floor_d = kDiagFloor * E.mu * G.diag_rest_max;
  s.guard = kEnergyGuard * E.mu * G.vol_total;
  s.buffer = E.dhat;
  s.buffer_out = P.outer_mult * E.dhat;
  if (threadIdx.x == 0) {
    S.vel = P.vel ? P.vel + E.voff : nullptr;
    // density / dt^2 of the dynamic form (0: quasi-static); an env's own density
    // (t2r_set_densities) replaces the option's
    S.iw = (P.vel && P.inertia_w > 0.0) ? (E.density > 0.0 ? E.density / (P.dt * P.dt) : P.inertia_w) : 0.0;
    S.dt = P.dt;
  }
  __syncthreads();
  s.armijo = P.armijo;
  s.pair_cap = E.pair_cap;
  s.fric_cap = E.fric_cap;
  s.outer_cap = E.outer_cap;
  s.L = P.lists + (&E - P.envs);
  s.xs_o = P.xsnap + E.snoff;
  s.xs_i = P.xsnap + E.snoff + 3 * (long long)G.n_sv;
  s.reculls = s.restarts = s.halvings = s.ncand = s.outer_builds = 0;
  s.fill = 0.0;
  s.evals = 0;
  s.max_evals = P.max_evals > 0 ? P.max_evals : (1ll << 62);
}


}  // namespace t2r

using namespace t2r;

// Two workgroups of 256 threads (or one of 512) per CU: 2 waves per SIMD, which
// the register budget of the fully inlined step allows without spilling.
// One load step of env e: the indenter moves from the env's previous pose to
// q1 in continuation substeps (each a PNCG solve), with friction lagged at the
// previous equilibrium. On overflow or infeasibility the state is rolled back
// and the previous pose kept. Counters accumulate into st; returns the status.
__device__ __forceinline__ int load_step(const StepParams& P, int e, Solver& s, Shared& S, const double q1[7],
                                         EnvStats& st) {
  View& V = s.V;
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const EnvDev& E = *V.E;
  const int n = 3 * G.n_v;
  T2R_G double* pose_prev = P.pose_prev + 7 * e;
  double q0[7], qpp[7];
  #pragma unroll
  for (int i = 0; i < 7; ++i) { q0[i] = pose_prev[i]; qpp[i] = P.pose_lag[7 * e + i]; }
  __syncthreads();  // every thread has read q_{s-2} before it is replaced
  // q_{s-1} of this load step (its friction lag pose), kept for the adjoint
  if (threadIdx.x < 7) P.pose_lag[7 * e + threadIdx.x] = q0[threadIdx.x];
  // Warm start: when this step continues the previous one's indenter motion,
  // solve from x_{s-1} + f (x_{s-1} - x_{s-2}) (the quasi-static counterpart
  // of the inertial predictor x + h v), f the ratio of this step's indenter
  // motion to the part of the previous one that moved the gel: all of it in
  // contact; if the previous step started out of contact (d_min >= dhat), its
  // motion less the gap it closed (d_min at its start minus d_min at its end).
  double fac = 0.0, m_prev = 0.0, m_cur = 0.0;
  bool cont = false;
  if (P.warm_start) {
    m_prev = ind_motion(qpp, q0, I.r_max);
    m_cur = ind_motion(q0, q1, I.r_max);
    double d1d2 = 0.0, d1 = 0.0, d2 = 0.0, qs = 0.0;
    for (int i = 3; i < 7; ++i) qs += q0[i] * q1[i];
    for (int i = 0; i < 7; ++i) {
      const double b = (i >= 3 && qs < 0.0) ? -q1[i] : q1[i];  // same quaternion hemisphere
      const double u = q0[i] - qpp[i], w = b - q0[i];
      d1d2 += u * w; d1 += u * u; d2 += w * w;
    }
    cont = m_prev > 0.0 && m_cur > 0.0 && d1d2 > 0.9 * sqrt(d1 * d2);
  }
  // keep x_{s-1} for the friction lag and for rollback (g1 holds x_{s-1} - x_{s-2})
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double xc = V.x[j], xo = V.xprev[j];
    V.xprev[j] = xc;
    if (cont) V.g1[j] = xc - xo;
  }
  // friction lag and starting distance at (x_{s-1}, q_{s-1}), from the outer
  // list kept since the last step (rebuilt here if the motion since it was
  // built exceeds its margin; in deterministic mode always, so that a step's
  // lists, and their order, depend on its starting state only)
  if (threadIdx.x == 0) {
    set_pose(S, I, q0);
    if (V.det) { s.L->valid_o = 0; s.L->valid_i = 0; }
  }
  __syncthreads();
  int status = 0;
  double dmin_start;
  if (!ensure_lists(s, V.x, 0.0)) {
    status |= kOverflow;
    dmin_start = 0.0;
  } else {
    const int mode = (E.mu_f > 0.0) ? 1 : 2;
    const unsigned long long t0 = tick();
    double dm = lag_from_outer(s, V.x, mode, E.mu_f);
    const int cnt = S.count, ov = S.overflow;
    dmin_start = block_min(dm, S);
    tock(S, 9, t0);
    V.nfric = (mode == 1) ? min(cnt, s.fric_cap) : 0;
    if (mode == 1) s.fill = fmax(s.fill, (double)cnt / s.fric_cap);
    if (ov) status |= kOverflow;
  }
  st.n_friction = V.nfric;
  {
    const double gap_prev = P.gap0[e];  // d_min at the start of the previous step (0: unknown)
    __syncthreads();                    // read by every thread before it is replaced
    if (threadIdx.x == 0) P.gap0[e] = dmin_start;
    if (cont) {
      const double closed = (gap_prev >= E.dhat && dmin_start > 0.0) ? fmax(0.0, gap_prev - dmin_start) : 0.0;
      fac = m_cur / fmax(m_prev - closed, 0.25 * m_prev);
    }
  }
  bool direct = false;  // the warm start is feasible at q_s: one solve, no intermediate poses
  if (fac > 0.0 && !(status & kOverflow) && dmin_start > 0.0) {
    // take the warm start only if it is feasible at q_{s-1}: J > 0 and d > 0
    for (int j = threadIdx.x; j < n; j += blockDim.x) V.x[j] = fma(fac, V.g1[j], V.xprev[j]);
    __syncthreads();
    int feas = 1;
    elem_eval(V, V.x, V.p, 0.0, V.g1, V.diag, *s.T, feas);
    double f1[1] = {feas ? 0.0 : 1.0};
    block_reduce<0, 1>(f1, S);
    bool ok = f1[0] == 0.0 && ensure_lists(s, V.x, 0.0);
    double dm = 0.0;
    if (ok) {
      int na = 0;
      dm = dmin_all(s, V.x, na);
      ok = dm > 0.0;
    }
    if (ok) {
      dmin_start = dm;
      if (threadIdx.x == 0) set_pose(S, I, q1);
      __syncthreads();
      if (ensure_lists(s, V.x, 0.0)) {
        int na = 0;
        direct = dmin_all(s, V.x, na) > 0.05 * E.dhat;
      }
      if (threadIdx.x == 0) set_pose(S, I, q0);
      __syncthreads();
    } else {
      for (int j = threadIdx.x; j < n; j += blockDim.x) V.x[j] = V.xprev[j];
      __syncthreads();
      if (!ensure_lists(s, V.x, 0.0)) status |= kOverflow;
    }
  }
  int status_acc = kConverged;
  double tau = 0.0, dmin = dmin_start;
  int sub = 0;
  double res = 0.0, energy = 0.0;
  int nact = 0;
  if (!(dmin_start > 0.0)) {
    status_acc = kInfeasible;
  } else {
    // continuation rate |dt| + theta r_max of the indenter's points
    double dt = 0.0;
    #pragma unroll
    for (int i = 0; i < 3; ++i) dt += (q1[i] - q0[i]) * (q1[i] - q0[i]);
    dt = sqrt(dt);
    double qa = 0.0, na = 0.0, nb = 0.0;
    for (int i = 3; i < 7; ++i) { qa += q0[i] * q1[i]; na += q0[i] * q0[i]; nb += q1[i] * q1[i]; }
    const double cth = fmin(1.0, fabs(qa) / sqrt(na * nb));
    const double theta = 2.0 * acos(cth);
    const double rate = dt + theta * I.r_max;
    while (tau < 1.0 && sub < P.max_substeps) {
      const double dtau = (rate > 0.0 && !direct) ? 0.5 * fmin(E.dhat, dmin) / rate : 1.0 - tau;
      const double tau_new = fmin(1.0, tau + dtau);
      if (threadIdx.x == 0) {
        double q[7];
        interp_pose(q0, q1, tau_new, q);
        set_pose(S, I, q);
      }
      __syncthreads();
      const bool last = tau_new >= 1.0;
      const double tol = (last || P.substep_tol <= 0.0) ? P.tol : fmax(P.tol, P.substep_tol);
      int iters = 0;
      const int stt = pncg(s, tol, P.max_iters, iters, res, energy, nact);
      st.iters += iters;
      st.max_solve_iters = max(st.max_solve_iters, iters);
      ++sub;
      tau = tau_new;
      if (stt & (kOverflow | kInfeasible)) { status_acc = stt; break; }
      if (stt & kBudget) { status_acc = stt; break; }  // the env stops: rolled back below
      if (!(stt & kConverged)) status_acc = (status_acc & ~kConverged) | stt;
      int na2 = 0;
      dmin = dmin_all(s, V.x, na2);
    }
    if (tau < 1.0 && !(status_acc & (kOverflow | kInfeasible | kBudget)))
      status_acc = (status_acc & ~kConverged) | kSubsteps;
  }
  status |= status_acc;
  if (status & (kOverflow | kInfeasible | kBudget)) {
    // roll back to x_{s-1}; the previous pose is kept
    for (int j = threadIdx.x; j < n; j += blockDim.x) V.x[j] = V.xprev[j];
    __syncthreads();
  } else {
    if (threadIdx.x == 0) {
      // the pose x is in equilibrium with: q1, or the last continuation pose
      // reached when max_substeps ended the step early (T2R_ENV_SUBSTEPS)
      double q[7];
      if (tau < 1.0) interp_pose(q0, q1, tau, q);
      #pragma unroll
      for (int i = 0; i < 7; ++i) pose_prev[i] = tau < 1.0 ? q[i] : q1[i];
    }
    if (S.iw > 0.0) {  // dynamic form: v = (x - x^t) / dt
      const double idt = 1.0 / S.dt;
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int v = j >= 2 * G.n_v ? j - 2 * G.n_v : (j >= G.n_v ? j - G.n_v : j);
        S.vel[j] = G.fixed[v] ? 0.0 : (V.x[j] - V.xprev[j]) * idt;
      }
    }
  }
  __syncthreads();
  {
    int na2 = 0;
    st.d_min = dmin_all(s, V.x, na2);
    st.n_active = na2;
  }
  st.substeps += sub;
  st.residual = res;
  st.energy = energy;
  return status;
}

// Marker displacements of env e at its current state into the output block of
// load step k.
__device__ __forceinline__ void write_markers(const StepParams& P, int k, const View& V) {
  if (!P.markers_out) return;
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  T2R_G double* mo = P.markers_out + (long long)k * P.markers_stride + 3 * V.E->moff;
  for (int m = threadIdx.x; m < G.n_m; m += blockDim.x) {
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
      double u = 0.0;
      #pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int v = G.marker_tri[j * G.n_m + m];
        u += G.marker_w[j * G.n_m + m] * (V.x[c * nv + v] - G.X[c * nv + v]);
      }
      mo[3 * m + c] = u;
    }
  }
}

// Every env advances through P.n_steps load steps (poses pose_in[k][env]).
// One workgroup owns one env for the whole launch; workgroups take envs in
// P.order (longest expected first).
// Two workgroups of 256 threads (or one of 512) per CU: 2 waves per SIMD.
// DET: deterministic mode as a compile-time constant, so that the atomic-mode
// instantiation carries none of its code.
template <int BLOCK, bool DET>
__global__ void __launch_bounds__(BLOCK, (BLOCK == 256 ? 2 : 1)) t2r_step_kernel(StepParams P) {
  __shared__ Shared S;
  __shared__ Tile T;
  const int e = P.order ? P.order[blockIdx.x] : (int)blockIdx.x;
  if (e >= P.n_env) return;
  Solver s;
  make_view(P, e, s.V);
  s.V.det = DET ? 1 : 0;
  View& V = s.V;
  init_solver(s, P, S, T);
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  const unsigned long long t_start = tick();
  if (threadIdx.x < 10) S.tacc[threadIdx.x] = 0ull;
  __syncthreads();
  EnvStats st;
  st.status = 0; st.iters = 0; st.substeps = 0; st.restarts = 0; st.halvings = 0; st.reculls = 0;
  st.n_candidates = 0; st.n_active = 0; st.n_friction = 0; st.max_solve_iters = 0;
  st.outer_builds = 0; st.n_outer = 0;
  st.d_min = kInf; st.residual = 0.0; st.energy = 0.0;
  for (int k = 0; k < 10; ++k) st.phase_ms[k] = 0.0;
  st.list_fill = 0.0;
  st.evals = 0; st.reserved = 0;
  const bool skip = P.env_mask && P.env_mask[e] == 0;
  load_lists(s);
  if (threadIdx.x < 7) S.qb[threadIdx.x] = P.pose_prev[7 * e + threadIdx.x];
  __syncthreads();
  for (int k = 0; k < P.n_steps; ++k) {
    double q1[7];
    target_pose(P, *V.E, e, k, S.qb, q1);
    bool bad = false;
    #pragma unroll
    for (int i = 0; i < 7; ++i) bad |= !isfinite(q1[i]);
    int status;
    if (skip || bad) {
      status = skip ? kSkipped : kNonFinite;
    } else {
      status = load_step(P, e, s, S, q1, st);
    }
    st.status = status;
    write_markers(P, k, V);
    if (P.tape_x) {
      const long long ent = (long long)P.tape_k0 + k + 1;
      T2R_G double* tx = P.tape_x + ent * P.tape_stride + V.E->voff;
      for (int j = threadIdx.x; j < 3 * nv; j += blockDim.x) tx[j] = V.x[j];
      if (threadIdx.x < 7) P.tape_q[(ent * P.n_env + e) * 7 + threadIdx.x] = P.pose_prev[7 * e + threadIdx.x];
    }
    if (threadIdx.x == 0 && P.status_out) P.status_out[(long long)k * P.n_env + e] = status;
  }
  st.restarts = s.restarts;
  st.halvings = s.halvings;
  st.reculls = s.reculls;
  st.outer_builds = s.outer_builds;
  st.n_candidates = s.ncand;
  st.n_outer = V.nouter;
  st.list_fill = s.fill;
  st.evals = (int)min(s.evals, (long long)INT32_MAX);
  if (P.x_out) {
    T2R_G double* xo = P.x_out + 3 * P.x_out_off[e];
    for (int j = threadIdx.x; j < 3 * nv; j += blockDim.x) {
      const int v = j / 3, c = j - 3 * v;
      xo[j] = V.x[c * nv + v];
    }
  }
  if (threadIdx.x == 0) {
    S.tacc[8] = wall_clock64() - t_start;
    for (int k = 0; k < 10; ++k) st.phase_ms[k] = (double)S.tacc[k] / P.clock_khz;
    P.stats[e] = st;
  }
}

// ---------------------------------------------------------------------------
// Adjoint: gradient of a marker loss at a frictionless equilibrium x*
// (implicit differentiation: H lambda = dL/dx, dL/dtheta = -lambda^T dg/dtheta;
// theta = E, nu, mu_f and a rigid pose offset). The solve is Jacobi-PCG with the
// exact Hessian applied matrix-free; all arithmetic is FP64.
// ---------------------------------------------------------------------------

// out = H_elastic v at x ([3][n_v]; every vertex written, fixed vertices 0).
__device__ __forceinline__ void elem_hvp(const View& V, const double* x, const double* v, double* out, Tile& T) {
  const GelDev& G = *V.G;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const int B = blockDim.x;
  const double mu = E.mu, lam = E.lam;
  for (int i = threadIdx.x; i < kTileVerts; i += B) {
#pragma unroll
    for (int c = 0; c < 3; ++c) T.g[c][i] = 0.0;
  }
  for (int tile = 0; tile < G.n_tiles; ++tile) {
    const int t0 = G.tile_tet[tile], t1 = G.tile_tet[tile + 1];
    SlotIdx cur;
    fetch_idx(G, tile, cur);
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
      if (cur.fl[s] >= 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T.x[c][threadIdx.x + s * B] = x[c * nv + cur.v[s]];
          T.p[c][threadIdx.x + s * B] = v[c * nv + cur.v[s]];
        }
    __syncthreads();
    for (int e = t0 + threadIdx.x; e < t1; e += B) {
      TetIn<false> t;
      load_tet<false>(G, e, t);
      int l[4];
      tet_ids(t.loc, l);
      double F[9], dF[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double f = 0.0, df = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            f += (T.x[a][l[k + 1]] - T.x[a][l[0]]) * t.Dm[k * 3 + b];
            df += (T.p[a][l[k + 1]] - T.p[a][l[0]]) * t.Dm[k * 3 + b];
          }
          F[a * 3 + b] = f;
          dF[a * 3 + b] = df;
        }
      double C[9];  // cofactor = J F^-T
      C[0] = F[4] * F[8] - F[5] * F[7];
      C[1] = F[5] * F[6] - F[3] * F[8];
      C[2] = F[3] * F[7] - F[4] * F[6];
      C[3] = F[2] * F[7] - F[1] * F[8];
      C[4] = F[0] * F[8] - F[2] * F[6];
      C[5] = F[1] * F[6] - F[0] * F[7];
      C[6] = F[1] * F[5] - F[2] * F[4];
      C[7] = F[2] * F[3] - F[0] * F[5];
      C[8] = F[0] * F[4] - F[1] * F[3];
      const double J = F[0] * C[0] + F[1] * C[1] + F[2] * C[2];
      const double iJ = 1.0 / J;
      const double lnJ = log(J);
      // A = F^-1 dF (F^-1 = C^T / J)
      double A[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          A[a * 3 + b] = (C[0 * 3 + a] * dF[0 * 3 + b] + C[1 * 3 + a] * dF[1 * 3 + b] +
                          C[2 * 3 + a] * dF[2 * 3 + b]) * iJ;
      const double trA = A[0] + A[4] + A[8];
      // dP = mu dF + (mu - lam lnJ) F^-T dF^T F^-T + lam tr(A) F^-T, with
      // (F^-T dF^T F^-T)_ab = (A F^-1)_ba = sum_k A_bk C_ak / J
      const double c1 = mu - lam * lnJ, c2 = lam * trA;
      double dP[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const double q = (A[b * 3 + 0] * C[a * 3 + 0] + A[b * 3 + 1] * C[a * 3 + 1] + A[b * 3 + 2] * C[a * 3 + 2]) * iJ;
          dP[a * 3 + b] = t.vol * (mu * dF[a * 3 + b] + c1 * q + c2 * C[a * 3 + b] * iJ);
        }
      double s0[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 1; i < 4; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double o = dP[a * 3 + 0] * t.Dm[(i - 1) * 3 + 0] + dP[a * 3 + 1] * t.Dm[(i - 1) * 3 + 1] +
                           dP[a * 3 + 2] * t.Dm[(i - 1) * 3 + 2];
          atomicAdd(&T.g[a][l[i]], o);
          s0[a] += o;
        }
#pragma unroll
      for (int a = 0; a < 3; ++a) atomicAdd(&T.g[a][l[0]], -s0[a]);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const int i = threadIdx.x + s * B;
      if (cur.fl[s] < 0) continue;
      const int vtx = cur.v[s];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double o = T.g[c][i];
        T.g[c][i] = 0.0;
        if (!(cur.fl[s] & kFirstTouch)) o += out[c * nv + vtx];
        if (cur.fl[s] & kFixedLast) o = 0.0;
        out[c * nv + vtx] = o;
      }
    }
    __syncthreads();
  }
}

// Thread partials of lambda^T g_mu and lambda^T g_lam, where the elastic
// gradient is mu g_mu + lam g_lam: sum_e V (F - F^-T) : dF and
// sum_e V ln J F^-T : dF with dF the deformation gradient of lambda.
__device__ __forceinline__ void elem_theta(const View& V, const double* x, const double* lv, Tile& T,
                                           double& c_mu, double& c_lam) {
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  const int B = blockDim.x;
  for (int tile = 0; tile < G.n_tiles; ++tile) {
    const int t0 = G.tile_tet[tile], t1 = G.tile_tet[tile + 1];
    SlotIdx cur;
    fetch_idx(G, tile, cur);
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
      if (cur.fl[s] >= 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T.x[c][threadIdx.x + s * B] = x[c * nv + cur.v[s]];
          T.p[c][threadIdx.x + s * B] = lv[c * nv + cur.v[s]];
        }
    __syncthreads();
    for (int e = t0 + threadIdx.x; e < t1; e += B) {
      TetIn<false> t;
      load_tet<false>(G, e, t);
      int l[4];
      tet_ids(t.loc, l);
      double F[9], dF[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double f = 0.0, df = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            f += (T.x[a][l[k + 1]] - T.x[a][l[0]]) * t.Dm[k * 3 + b];
            df += (T.p[a][l[k + 1]] - T.p[a][l[0]]) * t.Dm[k * 3 + b];
          }
          F[a * 3 + b] = f;
          dF[a * 3 + b] = df;
        }
      double C[9];
      C[0] = F[4] * F[8] - F[5] * F[7];
      C[1] = F[5] * F[6] - F[3] * F[8];
      C[2] = F[3] * F[7] - F[4] * F[6];
      C[3] = F[2] * F[7] - F[1] * F[8];
      C[4] = F[0] * F[8] - F[2] * F[6];
      C[5] = F[1] * F[6] - F[0] * F[7];
      C[6] = F[1] * F[5] - F[2] * F[4];
      C[7] = F[2] * F[3] - F[0] * F[5];
      C[8] = F[0] * F[4] - F[1] * F[3];
      const double J = F[0] * C[0] + F[1] * C[1] + F[2] * C[2];
      const double iJ = 1.0 / J;
      double fdf = 0.0, cdf = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        fdf += F[k] * dF[k];
        cdf += C[k] * dF[k];
      }
      c_mu += t.vol * (fdf - cdf * iJ);
      c_lam += t.vol * log(J) * cdf * iJ;
    }
    __syncthreads();
  }
}

// Barrier Hessian times v at x, added into gout (LDS sums: gq = v, gd = out).
template <bool LDS>
__device__ __forceinline__ void pairs_hvp(const View& V, const Shared& S, Tile& T, const double* x,
                                          const double* v, double* out) {
  const GelDev& G = *V.G;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const double dh = E.dhat, kap = E.kappa;
  for (int i = threadIdx.x; i < V.npairs; i += blockDim.x) {
    if (!(V.pd[i] < dh)) continue;
    int2 pr = make_int2(0, 0);
    uint64_t rec = 0;
    if constexpr (LDS) rec = V.pslot[i];
    else pr = V.pairs[i];
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    if (!(d > 0.0) || d >= dh) continue;
    double b, b1, b2;
    barrier3(d, dh, b, b1, b2);
    const double invd = 1.0 / d;
    const double n[3] = {r[0] * invd, r[1] * invd, r[2] * invd};
    double D[2][3];
    #pragma unroll
    for (int w = 0; w < 2; ++w)
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        D[w][c] = cw_of(f, 0, w) * P.z[0][c] + cw_of(f, 1, w) * P.z[1][c] + cw_of(f, 2, w) * P.z[2][c] + cw_of(f, 3, w) * P.z[3][c];
    double Mi[2][2];
    gram_inverse(D, f.k, Mi);
    double q[3] = {0, 0, 0}, vv[2] = {0, 0}, da[3] = {0, 0, 0}, db[3] = {0, 0, 0};
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = P.gid[k];
      if (g < 0) continue;
      double pk[3];
      #pragma unroll
      for (int c = 0; c < 3; ++c) pk[c] = LDS ? T.gq[c][g] : v[c * nv + g];
      #pragma unroll
      for (int c = 0; c < 3; ++c) q[c] += f.c[k] * pk[c];
      // v_1 - v_0 and v_3 - v_2 of an edge-edge pair (indenter points: v = 0)
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (k < 2) da[c] += k == 0 ? -pk[c] : pk[c];
        else db[c] += k == 2 ? -pk[c] : pk[c];
      }
      const double rp = dot3(r, pk);
      #pragma unroll
      for (int w = 0; w < 2; ++w) if (w < f.k) vv[w] += cw_of(f, k, w) * rp + f.c[k] * dot3(D[w], pk);
    }
    const double wv[2] = {Mi[0][0] * vv[0] + Mi[0][1] * vv[1], Mi[1][0] * vv[0] + Mi[1][1] * vv[1]};
    const double nq = dot3(n, q);
    EdgeMoll M;
    const bool mol = edge_moll<LDS>(V, pr, rec, P, M);
    // ga, gb: dc/da, dc/db; ha, hb: the a and b blocks of (d2c) (v_1 - v_0, v_3 - v_2)
    double ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0}, ha[3] = {0, 0, 0}, hbv[3] = {0, 0, 0}, cp = 0.0;
    if (mol) {
      const double ad = dot3(M.a, da), bd = dot3(M.b, da), ae = dot3(M.a, db), be = dot3(M.b, db);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ga[c] = 2.0 * (M.bb * M.a[c] - M.ab * M.b[c]);
        gb[c] = 2.0 * (M.aa * M.b[c] - M.ab * M.a[c]);
        ha[c] = 2.0 * (M.bb * da[c] - M.b[c] * bd) + 4.0 * M.a[c] * be - 2.0 * M.b[c] * ae - 2.0 * M.ab * db[c];
        hbv[c] = 2.0 * (M.aa * db[c] - M.a[c] * ae) + 4.0 * M.b[c] * ad - 2.0 * M.a[c] * bd - 2.0 * M.ab * da[c];
      }
      cp = dot3(ga, da) + dot3(gb, db);
    }
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = P.gid[k];
      if (g < 0) continue;
      if (!LDS && G.fixed[g]) continue;
      const double ci = f.c[k];
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        double hv = ci * q[c] - ci * n[c] * nq;
        #pragma unroll
        for (int w = 0; w < 2; ++w)
          if (w < f.k) hv -= (cw_of(f, k, w) * r[c] + ci * D[w][c]) * wv[w];
        double hb = b2 * nq * ci * n[c] + b1 * hv * invd;
        if (mol) {  // gel points: the first edge (k = 0, 1), and for a gel-gel pair the second (2, 3)
          const double sg = (k == 0 || k == 2) ? -1.0 : 1.0;
          const double gc = sg * (k < 2 ? ga[c] : gb[c]), hc = sg * (k < 2 ? ha[c] : hbv[c]);
          hb = M.m * hb + M.m1 * b1 * (cp * ci * n[c] + nq * gc) + M.m2 * b * cp * gc + M.m1 * b * hc;
        }
        const double o = kap * hb;
        if constexpr (LDS) atomicAdd(&T.gd[c][g], o);
        else atomicAdd(&out[c * nv + g], o);
      }
    }
  }
}

// Thread partials of lambda^T (d g / d theta_pose) over the barrier pairs for
// the six pose directions: translations e_a, and rotations e_a x (y - t) of
// the indenter points about the indenter origin t. LDS path: gq = lambda.
template <bool LDS>
__device__ __forceinline__ void pairs_pose(const View& V, const Shared& S, const Tile& T, const double* x,
                                           const double* lv, double acc[6]) {
  const EnvDev& E = *V.E;
  const int nv = V.G->n_v;
  const double dh = E.dhat, kap = E.kappa;
  for (int i = threadIdx.x; i < V.npairs; i += blockDim.x) {
    if (!(V.pd[i] < dh)) continue;
    int2 pr = make_int2(0, 0);
    uint64_t rec = 0;
    if constexpr (LDS) rec = V.pslot[i];
    else pr = V.pairs[i];
    PairPts P;
    get_pair<LDS>(V, S, T, pr, rec, x, nullptr, 0.0, P);
    Feature f;
    classify(P, f);
    double r[3];
    const double d = pair_distance(P, f, r);
    if (!(d > 0.0) || d >= dh) continue;
    double b, b1, b2;
    barrier3(d, dh, b, b1, b2);
    const double invd = 1.0 / d;
    const double n[3] = {r[0] * invd, r[1] * invd, r[2] * invd};
    double D[2][3];
    #pragma unroll
    for (int w = 0; w < 2; ++w)
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        D[w][c] = cw_of(f, 0, w) * P.z[0][c] + cw_of(f, 1, w) * P.z[1][c] + cw_of(f, 2, w) * P.z[2][c] + cw_of(f, 3, w) * P.z[3][c];
    double Mi[2][2];
    gram_inverse(D, f.k, Mi);
    // gel side (lambda)
    double q1[3] = {0, 0, 0}, v1[2] = {0, 0}, da[3] = {0, 0, 0};
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = P.gid[k];
      if (g < 0) continue;
      double pk[3];
      #pragma unroll
      for (int c = 0; c < 3; ++c) pk[c] = LDS ? T.gq[c][g] : lv[c * nv + g];
      #pragma unroll
      for (int c = 0; c < 3; ++c) q1[c] += f.c[k] * pk[c];
      if (k < 2) {  // lambda_1 - lambda_0 of an edge-edge pair's gel edge
        #pragma unroll
        for (int c = 0; c < 3; ++c) da[c] += k == 0 ? -pk[c] : pk[c];
      }
      const double rp = dot3(r, pk);
      #pragma unroll
      for (int w = 0; w < 2; ++w) if (w < f.k) v1[w] += cw_of(f, k, w) * rp + f.c[k] * dot3(D[w], pk);
    }
    const double n1 = dot3(n, q1);
    const double m1[2] = {Mi[0][0] * v1[0] + Mi[0][1] * v1[1], Mi[1][0] * v1[0] + Mi[1][1] * v1[1]};
    EdgeMoll M;
    const bool mol = edge_moll<LDS>(V, pr, rec, P, M);
    double c1 = 0.0, aD = 0.0, bD = 0.0;
    if (mol) {
      aD = dot3(M.a, da);
      bD = dot3(M.b, da);
      c1 = 2.0 * (M.bb * aD - M.ab * bD);   // grad c . lambda
    }
    #pragma unroll
    for (int a = 0; a < 6; ++a) {
      double q2[3] = {0, 0, 0}, v2[2] = {0, 0}, db[3] = {0, 0, 0};
      #pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (P.gid[k] >= 0) continue;
        double dy[3] = {0.0, 0.0, 0.0};
        if (a < 3) {
          dy[a] = 1.0;
        } else {
          double y[3];
          #pragma unroll
          for (int c = 0; c < 3; ++c) y[c] = P.z[k][c] - S.t[c];
          const int ax = a - 3;  // e_ax x y
          dy[0] = (ax == 1 ? y[2] : 0.0) - (ax == 2 ? y[1] : 0.0);
          dy[1] = (ax == 2 ? y[0] : 0.0) - (ax == 0 ? y[2] : 0.0);
          dy[2] = (ax == 0 ? y[1] : 0.0) - (ax == 1 ? y[0] : 0.0);
        }
        #pragma unroll
        for (int c = 0; c < 3; ++c) q2[c] += f.c[k] * dy[c];
        if (k >= 2) {  // dy_3 - dy_2 of an edge-edge pair's indenter edge
          #pragma unroll
          for (int c = 0; c < 3; ++c) db[c] += k == 2 ? -dy[c] : dy[c];
        }
        const double rp = dot3(r, dy);
        #pragma unroll
        for (int w = 0; w < 2; ++w) if (w < f.k) v2[w] += cw_of(f, k, w) * rp + f.c[k] * dot3(D[w], dy);
      }
      const double n2 = dot3(n, q2);
      const double hd = (dot3(q1, q2) - (m1[0] * v2[0] + m1[1] * v2[1])) * invd - n1 * n2 * invd;
      double hb = b2 * n1 * n2 + b1 * hd;
      if (mol) {
        const double ab2 = dot3(M.a, db), bb2 = dot3(M.b, db);
        const double c2 = 2.0 * (M.aa * bb2 - M.ab * ab2);                             // grad c . dy
        const double cx = 4.0 * aD * bb2 - 2.0 * bD * ab2 - 2.0 * M.ab * dot3(da, db);  // lambda^T (d2c/da db) dy
        hb = M.m * hb + M.m1 * b1 * (c1 * n2 + n1 * c2) + M.m2 * b * c1 * c2 + M.m1 * b * cx;
      }
      acc[a] += kap * hb;
    }
  }
}

// out += H_f v: Hessian-vector product of the lagged friction term (records
// carry mu_f lambda_k). LDS path: gx = x and gq = v at the gel slots, sums in gd.
template <bool LDS>
__device__ __forceinline__ void fric_hvp(const View& V, const Shared& S, Tile& T, const double* x,
                                         const double* v, double* out) {
  const GelDev& G = *V.G;
  const int nv = G.n_v;
  const double eps = V.E->eps_v;
  for (int i = threadIdx.x; i < V.nfric; i += blockDim.x) {
    const FricPair F = V.fric[i];
    double Dl[3];
    fric_delta<LDS>(V, S, T, F, x, nullptr, 0.0, Dl);
    const double nD = dot3(F.n, Dl);
    double TD[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) TD[c] = Dl[c] - nD * F.n[c];
    const double s = sqrt(dot3(TD, TD));
    double f, fos, corr;
    mollifier3(s, eps, f, fos, corr);
    double q[3] = {0, 0, 0};
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int vv = F.gv[k];
      if (vv < 0) continue;
      #pragma unroll
      for (int c = 0; c < 3; ++c) q[c] += F.a[k] * (LDS ? T.gq[c][fric_gslot(F, k)] : v[c * nv + vv]);
    }
    const double nq = dot3(F.n, q);
    double uh[3] = {0, 0, 0}, uq = 0.0;
    if (s > 0) {
      #pragma unroll
      for (int c = 0; c < 3; ++c) uh[c] = TD[c] / s;
      uq = dot3(uh, q);
    }
    double hq[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) hq[c] = F.mulam * (fos * (q[c] - nq * F.n[c]) + corr * uq * uh[c]);
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int vv = F.gv[k];
      if (vv < 0) continue;
      if (!LDS && G.fixed[vv]) continue;
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double o = F.a[k] * hq[c];
        if constexpr (LDS) atomicAdd(&T.gd[c][fric_gslot(F, k)], o);
        else atomicAdd(&out[c * nv + vv], o);
      }
    }
  }
}

// Friction terms of one load step of the adjoint, over the lag records (built
// at (x_{s-1}, q_{s-1}) with coefficient mrec lambda_k); S holds q_s. Adds
//   acc[0]   += lambda^T g_f / mu_f                     (d/d mu_f: unit coefficient)
//   acc[1+a] += lambda^T (d g_f / d y(q_s)) dy_a        (pose offset at q_s)
//   acc[1+a] += (d Q / d y(q_{s-1})) . dy_a             (pose offset at q_{s-1})
//   carry    -= d Q / d x_{s-1}                         (free gel vertices)
// with Q = lambda^T g_f and dy_a the pose directions (translations e_a,
// rotations e_a x (y - t) about the indenter origin t of that pose). Q depends
// on the lag points through lambda_k = -kappa b'(d), the normal n, the
// relative displacement and the closest-point weights c(w); the free
// parameters w move with the points by the implicit-function theorem on the
// closest-point optimality D^T r = 0: (D^T D) dw = -sum_i (Cw_i r + c_i D) dz_i.
// Global-memory path (one pass per load step).
__device__ __forceinline__ void fric_adjoint(const View& V, const Shared& S, Tile& T, const double* xs, const double* xp,
                             const double* lam, const double qp[7], double mrec, double acc[7],
                             double* carry) {
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const double eps = E.eps_v, dh = E.dhat, kap = E.kappa, muf = E.mu_f;
  double Rp[9];
  quat_to_R(qp + 3, Rp);
  for (int i = threadIdx.x; i < V.nfric; i += blockDim.x) {
    const FricPair F = V.fric[i];
    const double lamk = F.mulam / mrec;
    double Dl[3];
    fric_delta<false>(V, S, T, F, xs, nullptr, 0.0, Dl);
    const double nD0 = dot3(F.n, Dl);
    double TD[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) TD[c] = Dl[c] - nD0 * F.n[c];
    const double sl = sqrt(dot3(TD, TD));
    double f, fos, corr;
    mollifier3(sl, eps, f, fos, corr);
    double uh[3] = {0, 0, 0};
    if (sl > 0) {
      #pragma unroll
      for (int c = 0; c < 3; ++c) uh[c] = TD[c] / sl;
    }
    // d/d mu_f and q1 = sum a_k lambda_k
    double q1[3] = {0, 0, 0};
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int v = F.gv[k];
      if (v < 0) continue;
      double lk[3];
      #pragma unroll
      for (int c = 0; c < 3; ++c) { lk[c] = lam[c * nv + v]; q1[c] += F.a[k] * lk[c]; }
      acc[0] += lamk * F.a[k] * fos * dot3(TD, lk);
    }
    if (!(muf > 0.0)) continue;
    const double w = muf * lamk;
    // pose at q_s: the indenter points enter the relative displacement with -c_j
    {
      const double n1 = dot3(F.n, q1), u1 = dot3(uh, q1);
      #pragma unroll
      for (int a = 0; a < 6; ++a) {
        double q2[3] = {0, 0, 0};
        #pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (F.iv[k] < 0) continue;
          double y[3], dy[3] = {0, 0, 0};
          ind_world(S, I, F.iv[k], y);
          if (a < 3) {
            dy[a] = 1.0;
          } else {
            const int ax = a - 3;
            const double yr[3] = {y[0] - S.t[0], y[1] - S.t[1], y[2] - S.t[2]};
            dy[0] = (ax == 1 ? yr[2] : 0.0) - (ax == 2 ? yr[1] : 0.0);
            dy[1] = (ax == 2 ? yr[0] : 0.0) - (ax == 0 ? yr[2] : 0.0);
            dy[2] = (ax == 0 ? yr[1] : 0.0) - (ax == 1 ? yr[0] : 0.0);
          }
          #pragma unroll
          for (int c = 0; c < 3; ++c) q2[c] -= F.c[k] * dy[c];
        }
        acc[1 + a] += w * (fos * (dot3(q1, q2) - n1 * dot3(F.n, q2)) + corr * u1 * dot3(uh, q2));
      }
    }
    // the lag: points in the distance routine's order (make_fric keeps it)
    int ng = 0;
    #pragma unroll
    for (int k = 0; k < 3; ++k) ng += F.gv[k] >= 0 ? 1 : 0;
    PairPts P;
    P.kind = ng == 1 ? kVF : (ng == 3 ? kFV : kEE);
    double Z[4][3], L[4][3];
    int vid[4];
    {
      int jg = 0, ji = 0;
      #pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (point_is_gel(P.kind, k)) {
          const int v = F.gv[jg++];
          vid[k] = v;
          P.gid[k] = v;
          #pragma unroll
          for (int c = 0; c < 3; ++c) {
            P.z[k][c] = xp[c * nv + v];
            Z[k][c] = xs[c * nv + v];
            L[k][c] = lam[c * nv + v];
          }
        } else {
          const int j = F.iv[ji++];
          vid[k] = j;
          P.gid[k] = -1;
          const double a0 = I.Y[j], a1 = I.Y[I.n_v + j], a2 = I.Y[2 * I.n_v + j];
          double y[3];
          ind_world(S, I, j, y);
          #pragma unroll
          for (int c = 0; c < 3; ++c) {
            P.z[k][c] = Rp[c * 3 + 0] * a0 + Rp[c * 3 + 1] * a1 + Rp[c * 3 + 2] * a2 + qp[c];
            Z[k][c] = y[c];
            L[k][c] = 0.0;
          }
        }
      }
    }
    Feature fe;
    classify(P, fe);
    double r[3];
    const double d = pair_distance(P, fe, r);
    if (!(d > 0.0) || d >= dh) continue;
    const double sig = (P.kind == kFV) ? -1.0 : 1.0;
    double b, b1, b2;
    barrier3(d, dh, b, b1, b2);
    const double lamd = -kap * b1;
    double rh[3], nn[3], Dt[3] = {0, 0, 0}, Lb[3] = {0, 0, 0};
    #pragma unroll
    for (int c = 0; c < 3; ++c) { rh[c] = r[c] / d; nn[c] = sig * rh[c]; }
    #pragma unroll
    for (int k = 0; k < 4; ++k)
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        Dt[c] += sig * fe.c[k] * (Z[k][c] - P.z[k][c]);
        Lb[c] += fe.c[k] * L[k][c];
      }
    const double nD = dot3(nn, Dt);
    double u[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = Dt[c] - nD * nn[c];
    const double su = sqrt(dot3(u, u));
    double phi, dphi;
    if (su < eps) { phi = -su / (eps * eps) + 2.0 / eps; dphi = -1.0 / (eps * eps); }
    else { phi = 1.0 / su; dphi = -1.0 / (su * su); }
    const double Cq = sig * dot3(Lb, u);
    // reverse mode through Q = mu_f lambda(d) phi(|u|) C
    const double lam_b = muf * phi * Cq, phi_b = muf * lamd * Cq, C_b = muf * lamd * phi;
    const double d_b = lam_b * (-kap * b2);
    const double s_b = phi_b * dphi;
    double ub[3], Lbb[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
      ub[c] = C_b * sig * Lb[c] + (su > 0.0 ? s_b * u[c] / su : 0.0);
      Lbb[c] = C_b * sig * u[c];
    }
    const double nub = dot3(nn, ub);
    double Dtb[3], rb[3];
    #pragma unroll
    for (int c = 0; c < 3; ++c) Dtb[c] = ub[c] - nub * nn[c];
    {
      double rhb[3];
      #pragma unroll
      for (int c = 0; c < 3; ++c) rhb[c] = sig * (-nD * ub[c] - nub * Dt[c]);
      const double rr = dot3(rh, rhb);
      #pragma unroll
      for (int c = 0; c < 3; ++c) rb[c] = (rhb[c] - rr * rh[c]) / d + d_b * rh[c];
    }
    double cb[4], Zb[4][3];
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      double dz[3];
      #pragma unroll
      for (int c = 0; c < 3; ++c) dz[c] = Z[k][c] - P.z[k][c];
      cb[k] = sig * dot3(Dtb, dz) + dot3(Lbb, L[k]) + dot3(rb, P.z[k]);
      #pragma unroll
      for (int c = 0; c < 3; ++c) Zb[k][c] = (-sig * Dtb[c] + rb[c]) * fe.c[k];
    }
    // closest-point parameters
    double D[2][3];
    #pragma unroll
    for (int a = 0; a < 2; ++a)
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        D[a][c] = cw_of(fe, 0, a) * P.z[0][c] + cw_of(fe, 1, a) * P.z[1][c] + cw_of(fe, 2, a) * P.z[2][c] +
                  cw_of(fe, 3, a) * P.z[3][c];
    double Mi[2][2];
    gram_inverse(D, fe.k, Mi);
    double wb[2] = {0, 0};
    #pragma unroll
    for (int a = 0; a < 2; ++a)
      if (a < fe.k)
        #pragma unroll
        for (int k = 0; k < 4; ++k) wb[a] += cb[k] * cw_of(fe, k, a);
    const double m[2] = {Mi[0][0] * wb[0] + Mi[0][1] * wb[1], Mi[1][0] * wb[0] + Mi[1][1] * wb[1]};
    #pragma unroll
    for (int k = 0; k < 4; ++k)
      #pragma unroll
      for (int a = 0; a < 2; ++a)
        if (a < fe.k)
          #pragma unroll
          for (int c = 0; c < 3; ++c) Zb[k][c] -= (cw_of(fe, k, a) * r[c] + fe.c[k] * D[a][c]) * m[a];
    // scatter: gel points to the carry, indenter points to the pose offset at q_{s-1}
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (P.gid[k] >= 0) {
        const int v = vid[k];
        if (G.fixed[v]) continue;
        #pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&carry[c * nv + v], -Zb[k][c]);
      } else {
        const double yr[3] = {P.z[k][0] - qp[0], P.z[k][1] - qp[1], P.z[k][2] - qp[2]};
        #pragma unroll
        for (int a = 0; a < 3; ++a) acc[1 + a] += Zb[k][a];
        // e_ax x yr
        acc[4] += Zb[k][1] * (-yr[2]) + Zb[k][2] * yr[1];
        acc[5] += Zb[k][0] * yr[2] + Zb[k][2] * (-yr[0]);
        acc[6] += Zb[k][0] * (-yr[1]) + Zb[k][1] * yr[0];
      }
    }
  }
}

// out = H v at x (elastic + barrier + the friction records in V.nfric), fixed DOFs 0.
__device__ __forceinline__ void hess_vec(Solver& s, const double* x, const double* v, double* out) {
  View& V = s.V;
  elem_hvp(V, x, v, out, *s.T);
  if (V.slots_ok) {
    stage_points(V, *s.S, *s.T, x, v, 0.0, 1);
    Tile& T = *s.T;
    for (int i = threadIdx.x; i < V.nslots; i += blockDim.x) {
#pragma unroll
      for (int c = 0; c < 3; ++c) T.gd[c][i] = 0.0;
    }
    __syncthreads();
    pairs_hvp<true>(V, *s.S, T, x, v, out);
    fric_hvp<true>(V, *s.S, T, x, v, out);
    const GelDev& G = *V.G;
    const int nv = G.n_v;
    __syncthreads();
    for (int i = threadIdx.x; i < V.nslots; i += blockDim.x) {
      const int vtx = V.slot_v[i];
      if (G.fixed[vtx]) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) out[c * nv + vtx] += T.gd[c][i];
    }
  } else {
    __syncthreads();
    pairs_hvp<false>(V, *s.S, *s.T, x, v, out);
    fric_hvp<false>(V, *s.S, *s.T, x, v, out);
  }
  __syncthreads();
}

// Adjoint of the last P.bw_steps recorded load steps, last step first:
//   H_s lambda_s = W^T dL/du_s + carry_s,   carry_{s-1} = -(d g_s / d x_{s-1})^T lambda_s,
//   dL/dtheta = -sum_s lambda_s^T d g_s / d theta,
// with every state read from the tape. The env's own positions, poses and
// friction records are not changed; its neighbour lists are rebuilt as needed.
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK, (BLOCK == 256 ? 2 : 1)) t2r_backward_kernel(StepParams P) {
  __shared__ Shared S;
  __shared__ Tile T;
  const int e = blockIdx.x;
  if (e >= P.n_env) return;
  Solver s;
  make_view(P, e, s.V);
  s.V.det = 0;  // the adjoint keeps its atomic sums
  View& V = s.V;
  init_solver(s, P, S, T);
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  const int n = 3 * nv;
  EnvStats st;
  st.status = 0; st.iters = 0; st.substeps = 0; st.restarts = 0; st.halvings = 0; st.reculls = 0;
  st.n_candidates = 0; st.n_active = 0; st.n_friction = 0; st.max_solve_iters = 0;
  st.outer_builds = 0; st.n_outer = 0; st.d_min = 0.0; st.residual = 0.0; st.energy = 0.0;
  for (int k = 0; k < 10; ++k) st.phase_ms[k] = 0.0;
  st.list_fill = 0.0;
  st.evals = 0; st.reserved = 0;
  const unsigned long long t_start = tick();
  load_lists(s);
  const double muf = E.mu_f;
  const double mrec = muf > 0.0 ? muf : 1.0;  // coefficient the lag records are built with
  T2R_G double* Ad = P.adj + E.voff;
  for (int j = threadIdx.x; j < n; j += blockDim.x) V.g1[j] = 0.0;  // carry into the last step: none
  __syncthreads();
  // thread partials of lambda^T dg/dtheta: mu-, lambda-elastic, mu_f, pose (6)
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  bool ok = true;
  int status = kConverged;
  for (int w = 0; w < P.bw_steps && ok; ++w) {
    const long long k = (long long)P.bw_last - w;
    T2R_G double* xs = P.tape_x + k * P.tape_stride + E.voff;
    T2R_G double* xp = xs - P.tape_stride;
    double qs[7], qp[7];
    #pragma unroll
    for (int i = 0; i < 7; ++i) {
      qs[i] = P.tape_q[(k * P.n_env + e) * 7 + i];
      qp[i] = P.tape_q[((k - 1) * P.n_env + e) * 7 + i];
    }
    V.x = xs;
    V.xprev = xp;
    // friction records at the lag (x_{s-1}, q_{s-1})
    V.nfric = 0;
    if (threadIdx.x == 0) set_pose(S, I, qp);
    __syncthreads();
    ok = ensure_lists(s, xp, 0.0);
    int nfric = 0;
    if (ok) {
      lag_from_outer(s, xp, 1, mrec);
      nfric = min(S.count, s.fric_cap);
      ok = S.overflow == 0;
    }
    __syncthreads();
    V.nfric = nfric;  // kept while the lists may be rebuilt, so the records keep their slots
    if (threadIdx.x == 0) set_pose(S, I, qs);
    __syncthreads();
    if (ok) ok = ensure_lists(s, xs, 0.0);
    if (!ok) break;
    st.n_friction = max(st.n_friction, nfric);
    // rhs = carry + W^T dL/du_s (free DOFs) in g1, lambda = 0 in g0
    const T2R_G double* du = P.dL_du + (long long)(P.bw_steps - 1 - w) * P.markers_stride + 3 * E.moff;
    for (int m = threadIdx.x; m < G.n_m; m += blockDim.x) {
      #pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int v = G.marker_tri[t * G.n_m + m];
        const double wt = G.marker_w[t * G.n_m + m];
        #pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&V.g1[c * nv + v], wt * du[3 * m + c]);
      }
    }
    // Jacobi preconditioner at x_s (the gradient output is scratch)
    V.nfric = muf > 0.0 ? nfric : 0;
    int feas, nact;
    eval_all<false>(s, xs, V.p, 0.0, Ad, V.diag, feas, nact);
    double a2[2] = {0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const int v = j >= 2 * nv ? j - 2 * nv : (j >= nv ? j - nv : j);
      double r = V.g1[j];
      if (G.fixed[v]) { r = 0.0; V.g1[j] = 0.0; }
      const double Pj = 1.0 / fmax(V.diag[j], s.floor_d);
      V.diag[j] = Pj;
      V.g0[j] = 0.0;
      V.p[j] = Pj * r;
      a2[0] += r * Pj * r;
      a2[1] += r * r;
    }
    block_reduce<2, 0>(a2, S);
    double rz = a2[0];
    const double r0 = sqrt(a2[1]);
    double rn = r0;
    int it = 0;
    for (; it < P.max_iters && rn > P.cg_tol * r0 && r0 > 0.0; ++it) {
      hess_vec(s, xs, V.p, Ad);
      // the three vector passes below load kVecUnroll entries per thread and trip
      // before using them (same per-thread order of the sums as one per trip)
      const int B = blockDim.x;
      double c1[1] = {0.0};
      for (int j0 = threadIdx.x; j0 < n; j0 += kVecUnroll * B) {
        double pv[kVecUnroll], av[kVecUnroll];
#pragma unroll
        for (int u = 0; u < kVecUnroll; ++u) {
          const int j = min(j0 + u * B, n - 1);
          pv[u] = V.p[j];
          av[u] = Ad[j];
        }
#pragma unroll
        for (int u = 0; u < kVecUnroll; ++u)
          if (j0 + u * B < n) c1[0] += pv[u] * av[u];
      }
      block_reduce<1, 0>(c1, S);
      if (!(c1[0] > 0.0)) { status |= kNonFinite; break; }
      const double alpha = rz / c1[0];
      double c2[2] = {0.0, 0.0};
      for (int j0 = threadIdx.x; j0 < n; j0 += kVecUnroll * B) {
        double pv[kVecUnroll], xv[kVecUnroll], rv[kVecUnroll], av[kVecUnroll], dv[kVecUnroll];
#pragma unroll
        for (int u = 0; u < kVecUnroll; ++u) {
          const int j = min(j0 + u * B, n - 1);
          pv[u] = V.p[j];
          xv[u] = V.g0[j];
          rv[u] = V.g1[j];
          av[u] = Ad[j];
          dv[u] = V.diag[j];
        }
#pragma unroll
        for (int u = 0; u < kVecUnroll; ++u) {
          const int j = j0 + u * B;
          if (j < n) {
            V.g0[j] = fma(alpha, pv[u], xv[u]);
            const double r = rv[u] - alpha * av[u];
            V.g1[j] = r;
            c2[0] += r * dv[u] * r;
            c2[1] += r * r;
          }
        }
      }
      block_reduce<2, 0>(c2, S);
      const double beta = c2[0] / rz;
      rz = c2[0];
      rn = sqrt(c2[1]);
      for (int j0 = threadIdx.x; j0 < n; j0 += kVecUnroll * B) {
        double pv[kVecUnroll], dv[kVecUnroll], rv[kVecUnroll];
#pragma unroll
        for (int u = 0; u < kVecUnroll; ++u) {
          const int j = min(j0 + u * B, n - 1);
          pv[u] = V.p[j];
          dv[u] = V.diag[j];
          rv[u] = V.g1[j];
        }
#pragma unroll
        for (int u = 0; u < kVecUnroll; ++u) {
          const int j = j0 + u * B;
          if (j < n) V.p[j] = fma(beta, pv[u], dv[u] * rv[u]);
        }
      }
      __syncthreads();
    }
    st.iters += it;
    st.max_solve_iters = max(st.max_solve_iters, it);
    st.residual = fmax(st.residual, r0 > 0.0 ? rn / r0 : 0.0);
    if (!(rn <= P.cg_tol * r0) && r0 > 0.0) status |= kMaxIter;
    // lambda^T dg/dtheta: elastic and barrier terms
    elem_theta(V, xs, V.g0, T, acc[0], acc[1]);
    double pose_acc[6] = {0, 0, 0, 0, 0, 0};
    if (V.slots_ok) {
      stage_points(V, S, T, xs, V.g0, 0.0, 1);
      pairs_pose<true>(V, S, T, xs, V.g0, pose_acc);
    } else {
      pairs_pose<false>(V, S, T, xs, V.g0, pose_acc);
    }
    #pragma unroll
    for (int a = 0; a < 6; ++a) acc[3 + a] += pose_acc[a];
    // friction terms and the carry into step s-1 (g1 is free once the solve is done)
    V.nfric = nfric;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) V.g1[j] = 0.0;
    __syncthreads();
    double fa[7] = {0, 0, 0, 0, 0, 0, 0};
    fric_adjoint(V, S, T, xs, xp, V.g0, qp, mrec, fa, V.g1);
    acc[2] += fa[0];
    #pragma unroll
    for (int a = 0; a < 6; ++a) acc[3 + a] += fa[1 + a];
    __syncthreads();
  }
  double grad[9];
  for (int k = 0; k < 9; ++k) grad[k] = 0.0;
  block_reduce<3, 0>(acc, S);
  block_reduce<6, 0>(acc + 3, S);
  if (!ok) {
    status = kOverflow;
  } else {
    // Lame partials: mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu)(1 - 2 nu))
    const double mu = E.mu, lam = E.lam;
    const double Ey = mu * (3.0 * lam + 2.0 * mu) / (lam + mu);
    const double nu = lam / (2.0 * (lam + mu));
    const double dmu_dE = 1.0 / (2.0 * (1.0 + nu));
    const double dlam_dE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double dmu_dnu = -Ey / (2.0 * (1.0 + nu) * (1.0 + nu));
    const double dlam_dnu = Ey * (1.0 + 2.0 * nu * nu) / ((1.0 + nu) * (1.0 + nu) * (1.0 - 2.0 * nu) * (1.0 - 2.0 * nu));
    grad[0] = -(acc[0] * dmu_dE + acc[1] * dlam_dE);
    grad[1] = -(acc[0] * dmu_dnu + acc[1] * dlam_dnu);
    grad[2] = -acc[2];
    for (int k = 0; k < 6; ++k) grad[3 + k] = -acc[3 + k];
    if (E.has_off) {
      // the kernel's rotation gradient is for an incremental rotation d applied
      // after the env's offset exp(dw); exp([dw + e]x) = exp([J_l(dw) e]x) exp([dw]x)
      // to first order, so dL/d(dw) = J_l(dw)^T dL/dd
      const double* w = E.off + 3;
      const double a2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], a = sqrt(a2);
      const double c1 = a > 1e-6 ? (1.0 - cos(a)) / a2 : 0.5 - a2 / 24.0;
      const double c2 = a > 1e-6 ? (a - sin(a)) / (a2 * a) : 1.0 / 6.0 - a2 / 120.0;
      const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
      double J[9];
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
          double kk = 0.0;
          for (int m = 0; m < 3; ++m) kk += K[r * 3 + m] * K[m * 3 + cc];
          J[r * 3 + cc] = (r == cc ? 1.0 : 0.0) + c1 * K[r * 3 + cc] + c2 * kk;
        }
      double gr[3];
      for (int cc = 0; cc < 3; ++cc) gr[cc] = J[0 * 3 + cc] * grad[6] + J[1 * 3 + cc] * grad[7] + J[2 * 3 + cc] * grad[8];
      for (int cc = 0; cc < 3; ++cc) grad[6 + cc] = gr[cc];
    }
    if (status & (kMaxIter | kNonFinite)) status &= ~kConverged;
  }
  if (threadIdx.x < 9) P.grad_out[9 * e + threadIdx.x] = grad[threadIdx.x];
  if (threadIdx.x == 0) {
    st.status = status;
    st.n_candidates = V.npairs;
    st.n_outer = V.nouter;
    st.substeps = P.bw_steps;
    st.phase_ms[8] = (double)(wall_clock64() - t_start) / P.clock_khz;
    P.stats[e] = st;
  }
}

extern "C" hipError_t t2r_launch_backward(const StepParams* p, int block, hipStream_t stream) {
  if (block == 512)
    hipLaunchKernelGGL(t2r_backward_kernel<512>, dim3(p->n_env), dim3(512), 0, stream, *p);
  else if (block == 256)
    hipLaunchKernelGGL(t2r_backward_kernel<256>, dim3(p->n_env), dim3(256), 0, stream, *p);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Diagnostic evaluation of one env (state arrays are scratch copies).
__global__ void __launch_bounds__(256) t2r_eval_kernel(EvalParams Q) {
  __shared__ Shared S;
  __shared__ Tile T;
  const StepParams& P = Q.sp;
  Solver s;
  make_view(P, Q.env, s.V);
  View& V = s.V;
  init_solver(s, P, S, T);
  const GelDev& G = *V.G;
  const IndDev& I = *V.I;
  const EnvDev& E = *V.E;
  const int nv = G.n_v;
  load_lists(s);
  bool ok = true;
  if (Q.has_lag && E.mu_f > 0.0) {
    if (threadIdx.x == 0) set_pose(S, I, Q.pose_lag);
    __syncthreads();
    ok = ensure_lists(s, V.xprev, 0.0);
    if (ok) {
      lag_from_outer(s, V.xprev, 1, E.mu_f);
      V.nfric = min(S.count, s.fric_cap);
      ok = S.overflow == 0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) set_pose(S, I, Q.pose);
  __syncthreads();
  if (ok) ok = ensure_lists(s, V.x, 0.0);
  if (!ok) {
    // a list overflowed: report it instead of evaluating a truncated list
    if (threadIdx.x == 0) P.stats[0].status = kOverflow;
    return;
  }
  if (threadIdx.x == 0) P.stats[0].status = 0;
  int feas, nact;
  double eel = 0.0;
  const double Etot = eval_all<false>(s, V.x, V.p, 0.0, V.g0, V.diag, feas, nact, &eel);
  double curv = 0.0;
  if (Q.has_p) curv = curvature_all(s, V.x, V.p);
  int na2 = 0;
  const double dm = dmin_all(s, V.x, na2);
  for (int j = threadIdx.x; j < 3 * nv; j += blockDim.x) {
    const int v = j / 3, c = j - 3 * v;
    if (Q.grad_out) Q.grad_out[j] = V.g0[c * nv + v];
    if (Q.diag_out) Q.diag_out[j] = V.diag[c * nv + v];
  }
  if (threadIdx.x == 0 && Q.scalars_out) {
    Q.scalars_out[0] = Etot;
    Q.scalars_out[1] = curv;
    Q.scalars_out[2] = dm;
    Q.scalars_out[3] = (double)nact;
    Q.scalars_out[4] = feas ? 1.0 : 0.0;
    Q.scalars_out[5] = (double)V.npairs;
    Q.scalars_out[6] = (double)V.nfric;
    Q.scalars_out[7] = eel;
  }
}

// Converts between the ABI layout [n_v][3] and the state's [3][n_v] for every env.
// direction 0: in ([sum n_v][3] + 7 pose per env) -> state ; 1: state -> out.
__global__ void t2r_pack_kernel(StepParams P, const double* in, double* out, const long long* state_off,
                                int direction) {
  const int e = blockIdx.x;
  if (e >= P.n_env) return;
  const EnvDev& E = P.envs[e];
  const GelDev& G = P.gels[E.gel];
  const int nv = G.n_v;
  const long long base = state_off[e];
  if (direction == 0) {
    for (int j = threadIdx.x; j < 3 * nv; j += blockDim.x) {
      const int v = j / 3, c = j - 3 * v;
      P.x[E.voff + c * nv + v] = in[base + j];
    }
    if (threadIdx.x < 7) {
      P.pose_prev[7 * e + threadIdx.x] = in[base + 3 * nv + threadIdx.x];
      P.pose_lag[7 * e + threadIdx.x] = in[base + 3 * nv + threadIdx.x];  // no motion history
    }
  } else {
    for (int j = threadIdx.x; j < 3 * nv; j += blockDim.x) {
      const int v = j / 3, c = j - 3 * v;
      out[base + j] = P.x[E.voff + c * nv + v];
    }
    if (threadIdx.x < 7) out[base + 3 * nv + threadIdx.x] = P.pose_prev[7 * e + threadIdx.x];
  }
}

// Copies [n_v][3] (ABI layout) into [3][n_v] for one env's scratch slot.
__global__ void t2r_aos_to_soa_kernel(const double* in, double* out, int nv) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < 3 * nv; j += gridDim.x * blockDim.x) {
    const int v = j / 3, c = j - 3 * v;
    out[c * nv + v] = in[j];
  }
}

extern "C" hipError_t t2r_launch_step(const StepParams* p, int block, hipStream_t stream) {
  if (block == 512 && p->det)
    hipLaunchKernelGGL((t2r_step_kernel<512, true>), dim3(p->n_env), dim3(512), 0, stream, *p);
  else if (block == 256 && p->det)
    hipLaunchKernelGGL((t2r_step_kernel<256, true>), dim3(p->n_env), dim3(256), 0, stream, *p);
  else if (block == 512)
    hipLaunchKernelGGL((t2r_step_kernel<512, false>), dim3(p->n_env), dim3(512), 0, stream, *p);
  else if (block == 256)
    hipLaunchKernelGGL((t2r_step_kernel<256, false>), dim3(p->n_env), dim3(256), 0, stream, *p);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Longest-first env order. The expected cost of an env is the indenter motion
// of this launch (the summed bound |dt| + 2 sin(theta/2) r_max over its load
// steps) scaled by the square root of the env's previous cost per unit of
// motion (previous launch duration / its motion; 1 before the first launch).
// Bitonic sort of (cost, id) keys in LDS, one workgroup.
__global__ void __launch_bounds__(1024) t2r_order_kernel(StepParams P, int* order, double* motion) {
  __shared__ unsigned long long key[kOrderMax];
  const int n = P.n_env;
  if (n > kOrderMax) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) order[i] = i;
    return;
  }
  int np = 1;
  while (np < n) np <<= 1;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    unsigned long long k = ~0ull;
    if (i < n) {
      const double r_max = P.inds[P.envs[i].ind].r_max;
      double m = 0.0, q0[7], q1[7], qb[7];
      for (int c = 0; c < 7; ++c) q0[c] = qb[c] = P.pose_prev[7 * i + c];
      for (int s = 0; s < P.n_steps; ++s) {
        target_pose(P, P.envs[i], i, s, qb, q1);
        bool fin = true;
        for (int c = 0; c < 7; ++c) fin &= isfinite(q1[c]);
        if (!fin) continue;
        m += ind_motion(q0, q1, r_max);
        for (int c = 0; c < 7; ++c) q0[c] = q1[c];
      }
      const double ms = P.stats[i].phase_ms[8], pm = motion[i];
      const double rate = (ms > 0.0 && pm > 0.0 && isfinite(ms)) ? ms / pm : 1.0;
      motion[i] = m;
      const double cost = m * sqrt(rate);
      const float c = (cost > 0.0 && isfinite(cost)) ? (float)cost : 0.0f;
      // descending duration = ascending inverted bits (c >= 0), then ascending id
      k = ((unsigned long long)(~__float_as_uint(c)) << 32) | (unsigned)i;
    }
    key[i] = k;
  }
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long a = key[i], b = key[j];
          if ((a > b) == up) { key[i] = b; key[j] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) order[i] = (int)(key[i] & 0xffffffffu);
}

extern "C" hipError_t t2r_launch_order(const StepParams* p, int* order, double* motion, hipStream_t stream) {
  hipLaunchKernelGGL(t2r_order_kernel, dim3(1), dim3(1024), 0, stream, *p, order, motion);
  return hipGetLastError();
}

extern "C" hipError_t t2r_launch_eval(const EvalParams* q, int block, hipStream_t stream) {
  hipLaunchKernelGGL(t2r_eval_kernel, dim3(1), dim3(block), 0, stream, *q);
  return hipGetLastError();
}

extern "C" hipError_t t2r_launch_pack_state(const StepParams* p, const double* in, double* out,
                                            const long long* state_off, int direction, hipStream_t stream) {
  hipLaunchKernelGGL(t2r_pack_kernel, dim3(p->n_env), dim3(256), 0, stream, *p, in, out, state_off, direction);
  return hipGetLastError();
}

extern "C" hipError_t t2r_launch_aos_to_soa(const double* in, double* out, int nv, hipStream_t stream) {
  const int blocks = (3 * nv + 255) / 256;
  hipLaunchKernelGGL(t2r_aos_to_soa_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream, in, out, nv);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static workspace of t2r_backward_static: the two-entry trajectory tape
// (x_{s-1}, x_s and both poses) of a single-step adjoint, in a file-scope
// device array so that the call allocates nothing. Every GPU the library runs
// on holds its own copy until the process ends. In host code `scratch` names a
// host-side stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress) and only that address is ever handed to copies and
// kernels.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kStaticScratchDoubles = size_t(1) << 21;  // 16 MiB
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

// Device address and size (doubles) of `scratch` on `device`, which must be
// current. The first call on a device resolves the address; later calls reuse it.
extern "C" hipError_t t2r_static_scratch(int device, double** ptr, size_t* n_doubles) {
  static std::mutex lock;
  static double* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices || !ptr || !n_doubles) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<double*>(p);
  }
  *ptr = addr[device];
  *n_doubles = kStaticScratchDoubles;
  return hipSuccess;
}

extern "C" size_t t2r_static_scratch_capacity() { return kStaticScratchDoubles; }
