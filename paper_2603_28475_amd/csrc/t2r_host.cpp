// Host side of the t2r C ABI: argument validation, mesh preprocessing (rest
// shape, surface extraction, marker embedding, LDS tiles), indenter grids,
// device memory and kernel launches. See include/t2r.h for the contract.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/t2r.h"
#include "t2r_internal.h"

using namespace t2r;


namespace {

constexpr int kMaxVerts = 1 << 24;

struct GelHost {
  int n_v = 0, n_t = 0, n_m = 0;
  std::vector<double> X;          // [3][n_v]
  std::vector<uint8_t> fixed;
  // tiled tet data
  std::vector<int> tet;           // [4][n_t]
  std::vector<uint64_t> tet_local;
  std::vector<double> Dinv;       // [9][n_t]
  std::vector<double> vol;
  std::vector<float> Dinv32, vol32;
  std::vector<int> tile_tet, tile_vstart, tile_verts;
  std::vector<uint8_t> tile_flags;
  std::vector<int> surf_v, surf_e, surf_f;  // SoA
  std::vector<int> top_v;         // vertices of the top-face triangles (ascending)
  int n_sv = 0, n_se = 0, n_sf = 0, n_top = 0, n_fixed = 0;
  std::vector<int> marker_tri;    // [3][n_m]
  std::vector<double> marker_w;   // [3][n_m]
  double vol_total = 0.0, diag_rest_max = 0.0;
  GelDev dev{};
};

struct IndHost {
  int n_v = 0, n_f = 0, n_e = 0;
  std::vector<double> Y;          // [3][n_v]
  std::vector<int> tri;           // [3][n_f]
  std::vector<int> edge;          // [2][n_e]
  double r_max = 0.0, lo[3], hi[3];
  struct GridHost {
    double origin[3], inv_cell;
    int dims[3];
    std::vector<int> start, items;
    std::vector<double> box;      // [6][n]
    int n = 0;
  } gv, ge, gf;
  IndDev dev{};
};

struct EnvHost {
  int gel, ind;
  t2r_material mat;
  double pose0[7];
  int has_off = 0;
  double off[6] = {0, 0, 0, 0, 0, 0};  // rigid pose offset (dt, dw)
  double density = 0.0;                // own density of the dynamic form (0: the option's)
};

// pose0 moved by the env's rigid offset: q <- exp([dw]x) q (normalised),
// t <- t + dt (the same composition as the kernels' for every step pose)
void start_pose(const EnvHost& e, double out[7]) {
  for (int k = 0; k < 7; ++k) out[k] = e.pose0[k];
  if (!e.has_off) return;
  const double* w = e.off + 3;
  const double a = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double sc = a > 1e-12 ? sin(0.5 * a) / a : 0.5 - a * a / 48.0;
  const double ex[4] = {cos(0.5 * a), sc * w[0], sc * w[1], sc * w[2]};
  double qn = 0.0;
  for (int k = 3; k < 7; ++k) qn += e.pose0[k] * e.pose0[k];
  qn = sqrt(qn);
  const double q[4] = {e.pose0[3] / qn, e.pose0[4] / qn, e.pose0[5] / qn, e.pose0[6] / qn};
  out[3] = ex[0] * q[0] - ex[1] * q[1] - ex[2] * q[2] - ex[3] * q[3];
  out[4] = ex[0] * q[1] + ex[1] * q[0] + ex[2] * q[3] - ex[3] * q[2];
  out[5] = ex[0] * q[2] - ex[1] * q[3] + ex[2] * q[0] + ex[3] * q[1];
  out[6] = ex[0] * q[3] + ex[1] * q[2] - ex[2] * q[1] + ex[3] * q[0];
  for (int k = 0; k < 3; ++k) out[k] = e.pose0[k] + e.off[k];
}

}  // namespace

struct t2r_ctx {
  t2r_solver_opts opts;
  hipStream_t stream = nullptr;
  t2r_alloc_fn alloc = nullptr;
  t2r_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  std::string err;
  std::vector<GelHost> gels;
  std::vector<IndHost> inds;
  std::vector<EnvHost> envs;
  bool committed = false;
  std::vector<void*> allocs;
  // device arrays
  GelDev* d_gels = nullptr;
  IndDev* d_inds = nullptr;
  EnvDev* d_envs = nullptr;
  std::vector<EnvDev> h_envs;
  double *d_x = nullptr, *d_xprev = nullptr, *d_g0 = nullptr, *d_g1 = nullptr, *d_diag = nullptr,
         *d_p = nullptr, *d_pose_prev = nullptr;
  int2* d_pairs = nullptr;
  double* d_pair_d = nullptr;
  int2* d_outer = nullptr;
  ListState* d_lists = nullptr;
  double* d_xsnap = nullptr;
  FricPair* d_fric = nullptr;
  int* d_vmap = nullptr;
  int* d_imap = nullptr;
  int* d_islot_v = nullptr;
  int* d_order = nullptr;
  double* d_motion = nullptr;
  double* d_pose_lag = nullptr;
  double* d_adj = nullptr;
  double* d_gap = nullptr;  // [n_env] d_min at the start of each env's previous load step
  double* d_vel = nullptr;  // [sum 3 n_v] velocities of the dynamic form
  bool stepped = false;
  // trajectory tape (t2r_record): tape_cap recorded steps at most, tape_len so far
  double *d_tape_x = nullptr, *d_tape_q = nullptr;
  int tape_cap = 0, tape_len = 0;
  // bumped whenever a launch's parameters or device buffers change (allocation,
  // relayout, options, tape, materials): a captured launch is stale after a bump
  int64_t layout_gen = 0;
  // two-entry tape of the single-step adjoint (x_{s-1}, x_s)
  double *d_bw_x = nullptr, *d_bw_q = nullptr;
  uint64_t* d_oslot = nullptr;
  uint64_t* d_pslot = nullptr;
  int* d_slot_v = nullptr;
  EnvStats* d_stats = nullptr;
  long long* d_xout_off = nullptr;
  long long* d_state_off = nullptr;
  long long total_dofs = 0, total_verts = 0, total_markers = 0, state_size = 0;
  int pair_cap = 0;
  double clock_khz = 1.0;
  int n_cu = 256;      // compute units of the device (set at the first GPU call)
  int device = -1;     // the device current at the first GPU call
};

namespace {

t2r_status fail(t2r_ctx* c, t2r_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, call)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(ctx, T2R_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void* dev_alloc(t2r_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (c->alloc) {
    p = c->alloc(bytes, c->alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->allocs.push_back(p);
  return p;
}

void dev_free(t2r_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i) {
    if (c->allocs[i] == p) {
      if (c->free_fn) c->free_fn(p, c->alloc_user);
      else (void)hipFree(p);
      c->allocs.erase(c->allocs.begin() + (long)i);
      return;
    }
  }
}

void dev_free_all(t2r_ctx* c) {
  for (void* p : c->allocs) {
    if (c->free_fn) c->free_fn(p, c->alloc_user);
    else (void)hipFree(p);
  }
  c->allocs.clear();
}

template <typename T>
t2r_status upload(t2r_ctx* c, const std::vector<T>& v, const T** out) {
  T* p = (T*)dev_alloc(c, v.size() * sizeof(T));
  if (!p) return fail(c, T2R_E_NOMEM, "device allocation of %zu bytes failed", v.size() * sizeof(T));
  if (!v.empty()) HIP_TRY(c, hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  *out = p;
  return T2R_OK;
}

double det3(const double m[9]) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}

void inv3(const double m[9], double out[9]) {
  const double d = det3(m);
  out[0] = (m[4] * m[8] - m[5] * m[7]) / d;
  out[1] = (m[2] * m[7] - m[1] * m[8]) / d;
  out[2] = (m[1] * m[5] - m[2] * m[4]) / d;
  out[3] = (m[5] * m[6] - m[3] * m[8]) / d;
  out[4] = (m[0] * m[8] - m[2] * m[6]) / d;
  out[5] = (m[2] * m[3] - m[0] * m[5]) / d;
  out[6] = (m[3] * m[7] - m[4] * m[6]) / d;
  out[7] = (m[1] * m[6] - m[0] * m[7]) / d;
  out[8] = (m[0] * m[4] - m[1] * m[3]) / d;
}

uint32_t spread10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

struct Key3 {
  int a, b, c;
  bool operator==(const Key3& o) const { return a == o.a && b == o.b && c == o.c; }
};
struct Key3Hash {
  size_t operator()(const Key3& k) const {
    return ((size_t)k.a * 73856093u) ^ ((size_t)k.b * 19349663u) ^ ((size_t)k.c * 83492791u);
  }
};

// Builds the uniform grid of one primitive set (boxes given per primitive).
void build_grid(IndHost::GridHost& G, const std::vector<std::array<double, 6>>& boxes, const double lo[3],
                const double hi[3], double cell) {
  G.n = (int)boxes.size();
  for (int a = 0; a < 3; ++a) {
    G.origin[a] = lo[a] - 1e-9 * (1.0 + fabs(lo[a]));
    const double ext = hi[a] + 1e-9 * (1.0 + fabs(hi[a])) - G.origin[a];
    G.dims[a] = std::max(1, std::min(96, (int)ceil(ext / cell)));
  }
  // one inverse cell size for all axes: cover the largest extent
  double cmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double ext = hi[a] + 1e-9 * (1.0 + fabs(hi[a])) - G.origin[a];
    cmax = std::max(cmax, ext / G.dims[a]);
  }
  G.inv_cell = 1.0 / cmax;
  for (int a = 0; a < 3; ++a) {
    const double ext = hi[a] + 1e-9 * (1.0 + fabs(hi[a])) - G.origin[a];
    G.dims[a] = std::max(1, (int)ceil(ext * G.inv_cell));
  }
  auto cell_of = [&](double v, int a) {
    int c = (int)floor((v - G.origin[a]) * G.inv_cell);
    return c < 0 ? 0 : (c >= G.dims[a] ? G.dims[a] - 1 : c);
  };
  const int ncell = G.dims[0] * G.dims[1] * G.dims[2];
  std::vector<std::vector<int>> cells(ncell);
  G.box.assign(6 * (size_t)G.n, 0.0);
  for (int i = 0; i < G.n; ++i) {
    for (int k = 0; k < 6; ++k) G.box[(size_t)k * G.n + i] = boxes[i][k];
    int c0[3], c1[3];
    for (int a = 0; a < 3; ++a) { c0[a] = cell_of(boxes[i][a], a); c1[a] = cell_of(boxes[i][3 + a], a); }
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) cells[(z * G.dims[1] + y) * G.dims[0] + x].push_back(i);
  }
  G.start.assign(ncell + 1, 0);
  for (int k = 0; k < ncell; ++k) G.start[k + 1] = G.start[k] + (int)cells[k].size();
  G.items.clear();
  G.items.reserve(G.start[ncell]);
  for (auto& v : cells) G.items.insert(G.items.end(), v.begin(), v.end());
}

t2r_status commit(t2r_ctx* c);
t2r_status relayout_lists(t2r_ctx* c);
int pair_cap_of(const t2r_ctx* c, const GelHost& g);
template <typename T>
T* alloc_n(t2r_ctx* c, size_t n);

// Restarts the recording from the current state of every env (tape entry 0).
t2r_status tape_seed(t2r_ctx* c) {
  c->tape_len = 0;
  if (!c->d_tape_x) return T2R_OK;
  if (hipMemcpyAsync(c->d_tape_x, c->d_x, (size_t)c->total_dofs * sizeof(double), hipMemcpyDeviceToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(c->d_tape_q, c->d_pose_prev, 7 * c->envs.size() * sizeof(double), hipMemcpyDeviceToDevice,
                     c->stream) != hipSuccess)
    return fail(c, T2R_E_HIP, "tape copy failed");
  return T2R_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

void t2r_default_opts(t2r_solver_opts* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->substep_tol = 1e-4;
  o->max_iters = 20000;
  o->max_substeps = 1000;
  o->precision = 0;
  o->pair_capacity = 0;
  o->armijo = 1;
  o->block_size = 0;
  o->warm_start = 1;
  o->dynamic = 0;
  o->dt = 1.0 / 60.0;
  o->density = 1.1e-9;
  o->max_evals = 200000;
  o->ee_mollifier = 0;
  o->outer_radius = 0.0;
  o->deterministic = 0;
  o->self_contact = 0;
}

static t2r_status check_opts(t2r_ctx* c, const t2r_solver_opts* o) {
  if (!(o->tol > 0.0) || !isfinite(o->tol)) return fail(c, T2R_E_ARG, "tol must be positive");
  if (!isfinite(o->substep_tol)) return fail(c, T2R_E_ARG, "substep_tol must be finite");
  if (o->max_iters < 0 || o->max_substeps < 1) return fail(c, T2R_E_ARG, "max_iters >= 0 and max_substeps >= 1 required");
  if (o->precision != 0 && o->precision != 1) return fail(c, T2R_E_ARG, "precision must be 0 or 1");
  if (o->pair_capacity < 0) return fail(c, T2R_E_ARG, "pair_capacity must be >= 0");
  if (o->max_evals < 0) return fail(c, T2R_E_ARG, "max_evals must be >= 0 (0: no limit)");
  if (o->ee_mollifier != 0 && o->ee_mollifier != 1) return fail(c, T2R_E_ARG, "ee_mollifier must be 0 or 1");
  if (o->deterministic != 0 && o->deterministic != 1) return fail(c, T2R_E_ARG, "deterministic must be 0 or 1");
  if (o->self_contact != 0 && o->self_contact != 1) return fail(c, T2R_E_ARG, "self_contact must be 0 or 1");
  if (!(o->outer_radius == 0.0 || (o->outer_radius >= 2.0 && o->outer_radius <= 64.0)))
    return fail(c, T2R_E_ARG, "outer_radius must be 0 or in [2, 64] (got %g)", o->outer_radius);
  if (o->block_size != 0 && o->block_size != 256 && o->block_size != 512)
    return fail(c, T2R_E_ARG, "block_size must be 0 (256), 256 or 512");
  if (o->warm_start != 0 && o->warm_start != 1) return fail(c, T2R_E_ARG, "warm_start must be 0 or 1");
  if (o->dynamic != 0 && o->dynamic != 1) return fail(c, T2R_E_ARG, "dynamic must be 0 or 1");
  if (o->dynamic && (!(o->dt > 0.0) || !isfinite(o->dt) || !(o->density > 0.0) || !isfinite(o->density)))
    return fail(c, T2R_E_ARG, "the dynamic form needs dt > 0 and density > 0");
  return T2R_OK;
}

t2r_status t2r_create(t2r_ctx** out, const t2r_solver_opts* opts, void* hip_stream) {
  if (!out) return T2R_E_ARG;
  *out = nullptr;
  t2r_ctx* c = new (std::nothrow) t2r_ctx();
  if (!c) return T2R_E_NOMEM;
  t2r_default_opts(&c->opts);
  if (opts) {
    t2r_status s = check_opts(c, opts);
    if (s != T2R_OK) { delete c; return s; }
    c->opts = *opts;
  }
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return T2R_OK;
}

void t2r_destroy(t2r_ctx* c) {
  if (!c) return;
  if (c->committed) (void)hipStreamSynchronize(c->stream);
  dev_free_all(c);
  delete c;
}

const char* t2r_last_error(const t2r_ctx* c) { return c ? c->err.c_str() : "null context"; }

t2r_status t2r_set_allocator(t2r_ctx* c, t2r_alloc_fn a, t2r_free_fn f, void* user) {
  if (!c) return T2R_E_ARG;
  if (c->committed) return fail(c, T2R_E_STATE, "allocator must be set before the first GPU call");
  if ((a == nullptr) != (f == nullptr)) return fail(c, T2R_E_ARG, "alloc and free must both be set or both NULL");
  c->alloc = a;
  c->free_fn = f;
  c->alloc_user = user;
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_add_gel(t2r_ctx* c, int32_t n_v, const double* X, int32_t n_t, const int32_t* tets,
                       const uint8_t* fixed, int32_t n_m, const double* markers, int32_t* gel_id) {
  if (!c) return T2R_E_ARG;
  if (c->committed) return fail(c, T2R_E_STATE, "cannot add a gel after the first GPU call");
  if (n_v < 4 || n_v > kMaxVerts || n_t < 1 || n_t > 6 * kMaxVerts || n_m < 0)
    return fail(c, T2R_E_ARG, "bad sizes n_v=%d n_t=%d n_m=%d", n_v, n_t, n_m);
  if (!X || !tets || !fixed || (n_m > 0 && !markers) || !gel_id) return fail(c, T2R_E_ARG, "null pointer");
  GelHost g;
  g.n_v = n_v;
  g.n_t = n_t;
  g.n_m = n_m;
  g.X.resize(3 * (size_t)n_v);
  g.fixed.assign(fixed, fixed + n_v);
  for (int v = 0; v < n_v; ++v) {
    for (int a = 0; a < 3; ++a) {
      const double xv = X[3 * (size_t)v + a];
      if (!isfinite(xv)) return fail(c, T2R_E_ARG, "non-finite rest position at vertex %d", v);
      g.X[(size_t)a * n_v + v] = xv;
    }
    g.n_fixed += fixed[v] ? 1 : 0;
    if (fixed[v] > 1) return fail(c, T2R_E_ARG, "fixed flags must be 0 or 1");
  }
  std::vector<int> used(n_v, 0);
  std::vector<double> Dinv(9 * (size_t)n_t), vol(n_t);
  double xlo[3] = {1e300, 1e300, 1e300}, xhi[3] = {-1e300, -1e300, -1e300};
  for (int v = 0; v < n_v; ++v)
    for (int a = 0; a < 3; ++a) { xlo[a] = std::min(xlo[a], X[3 * v + a]); xhi[a] = std::max(xhi[a], X[3 * v + a]); }
  const double scale = std::max({xhi[0] - xlo[0], xhi[1] - xlo[1], xhi[2] - xlo[2], 1e-300});
  for (int e = 0; e < n_t; ++e) {
    int id[4];
    for (int k = 0; k < 4; ++k) {
      id[k] = tets[4 * (size_t)e + k];
      if (id[k] < 0 || id[k] >= n_v) return fail(c, T2R_E_ARG, "tet %d has vertex id %d out of range", e, id[k]);
      used[id[k]] = 1;
    }
    double Dm[9];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) Dm[a * 3 + k] = X[3 * (size_t)id[k + 1] + a] - X[3 * (size_t)id[0] + a];
    const double det = det3(Dm);
    if (!(det > 1e-12 * scale * scale * scale * 1e-6))
      return fail(c, T2R_E_ARG, "tet %d is inverted or degenerate (6V = %g)", e, det);
    inv3(Dm, &Dinv[9 * (size_t)e]);
    vol[e] = det / 6.0;
    g.vol_total += vol[e];
  }
  for (int v = 0; v < n_v; ++v)
    if (!used[v]) return fail(c, T2R_E_ARG, "vertex %d belongs to no tet", v);
  // rest diagonal scale: max_v sum_e V_e |g_i|^2
  {
    std::vector<double> dsum(n_v, 0.0);
    for (int e = 0; e < n_t; ++e) {
      const double* D = &Dinv[9 * (size_t)e];
      double g[4][3];
      for (int b = 0; b < 3; ++b) {
        g[1][b] = D[0 * 3 + b]; g[2][b] = D[1 * 3 + b]; g[3][b] = D[2 * 3 + b];
        g[0][b] = -(g[1][b] + g[2][b] + g[3][b]);
      }
      for (int k = 0; k < 4; ++k)
        dsum[tets[4 * (size_t)e + k]] += vol[e] * (g[k][0] * g[k][0] + g[k][1] * g[k][1] + g[k][2] * g[k][2]);
    }
    for (int v = 0; v < n_v; ++v)
      if (!fixed[v]) g.diag_rest_max = std::max(g.diag_rest_max, dsum[v]);
    if (g.diag_rest_max == 0.0) g.diag_rest_max = 1.0;
  }
  // surface: faces used by exactly one tet, outward by the opposite-vertex rule
  std::vector<std::array<int, 3>> btris;
  {
    std::unordered_map<Key3, std::pair<int, std::array<int, 3>>, Key3Hash> faces;
    faces.reserve(4 * (size_t)n_t);
    static const int lf[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    for (int e = 0; e < n_t; ++e) {
      for (int f = 0; f < 4; ++f) {
        std::array<int, 3> t = {tets[4 * (size_t)e + lf[f][0]], tets[4 * (size_t)e + lf[f][1]],
                                tets[4 * (size_t)e + lf[f][2]]};
        std::array<int, 3> s = t;
        std::sort(s.begin(), s.end());
        Key3 k{s[0], s[1], s[2]};
        auto it = faces.find(k);
        if (it == faces.end()) faces.emplace(k, std::make_pair(1, t));
        else it->second.first += 1;
      }
    }
    for (auto& kv : faces)
      if (kv.second.first == 1) btris.push_back(kv.second.second);
    std::sort(btris.begin(), btris.end(), [](const std::array<int, 3>& a, const std::array<int, 3>& b) {
      std::array<int, 3> sa = a, sb = b;
      std::sort(sa.begin(), sa.end());
      std::sort(sb.begin(), sb.end());
      return sa < sb;
    });
  }
  std::vector<std::array<int, 3>> stris;
  std::vector<std::pair<int, int>> sedges;
  std::vector<int> sverts;
  {
    std::vector<uint8_t> onb(n_v, 0);
    std::vector<std::pair<int, int>> es;
    for (auto& t : btris) {
      for (int k = 0; k < 3; ++k) {
        onb[t[k]] = 1;
        int a = t[k], b = t[(k + 1) % 3];
        es.push_back({std::min(a, b), std::max(a, b)});
      }
      if (!(fixed[t[0]] && fixed[t[1]] && fixed[t[2]])) stris.push_back(t);
    }
    std::sort(es.begin(), es.end());
    es.erase(std::unique(es.begin(), es.end()), es.end());
    for (auto& e : es)
      if (!(fixed[e.first] && fixed[e.second])) sedges.push_back(e);
    for (int v = 0; v < n_v; ++v)
      if (onb[v] && !fixed[v]) sverts.push_back(v);
  }
  g.n_sv = (int)sverts.size();
  g.n_se = (int)sedges.size();
  g.n_sf = (int)stris.size();
  g.surf_v = sverts;
  g.surf_e.resize(2 * (size_t)g.n_se);
  for (int i = 0; i < g.n_se; ++i) { g.surf_e[i] = sedges[i].first; g.surf_e[g.n_se + i] = sedges[i].second; }
  g.surf_f.resize(3 * (size_t)g.n_sf);
  for (int i = 0; i < g.n_sf; ++i)
    for (int k = 0; k < 3; ++k) g.surf_f[(size_t)k * g.n_sf + i] = stris[i][k];
  // markers: barycentric in the top-face triangle containing the rest xy
  {
    const double ztop = xhi[2];
    const double ztol = 1e-9 * (1.0 + fabs(ztop));
    std::vector<std::array<int, 3>> top;
    for (auto& t : stris)
      if (fabs(X[3 * (size_t)t[0] + 2] - ztop) <= ztol && fabs(X[3 * (size_t)t[1] + 2] - ztop) <= ztol &&
          fabs(X[3 * (size_t)t[2] + 2] - ztop) <= ztol)
        top.push_back(t);
    g.n_top = (int)top.size();
    for (auto& t : top) g.top_v.insert(g.top_v.end(), t.begin(), t.end());
    std::sort(g.top_v.begin(), g.top_v.end());
    g.top_v.erase(std::unique(g.top_v.begin(), g.top_v.end()), g.top_v.end());
    g.marker_tri.resize(3 * (size_t)n_m);
    g.marker_w.resize(3 * (size_t)n_m);
    for (int m = 0; m < n_m; ++m) {
      const double mx = markers[2 * (size_t)m], my = markers[2 * (size_t)m + 1];
      if (!isfinite(mx) || !isfinite(my)) return fail(c, T2R_E_ARG, "non-finite marker %d", m);
      bool found = false;
      for (auto& t : top) {
        const double ax = X[3 * (size_t)t[0]], ay = X[3 * (size_t)t[0] + 1];
        const double e1x = X[3 * (size_t)t[1]] - ax, e1y = X[3 * (size_t)t[1] + 1] - ay;
        const double e2x = X[3 * (size_t)t[2]] - ax, e2y = X[3 * (size_t)t[2] + 1] - ay;
        const double den = e1x * e2y - e1y * e2x;
        if (den == 0.0) continue;
        const double px = mx - ax, py = my - ay;
        const double s = (px * e2y - py * e2x) / den;
        const double r = (e1x * py - e1y * px) / den;
        const double w0 = 1.0 - s - r;
        if (w0 >= -1e-12 && s >= -1e-12 && r >= -1e-12) {
          for (int k = 0; k < 3; ++k) g.marker_tri[(size_t)k * n_m + m] = t[k];
          g.marker_w[m] = w0;
          g.marker_w[n_m + m] = s;
          g.marker_w[2 * (size_t)n_m + m] = r;
          found = true;
          break;
        }
      }
      if (!found) return fail(c, T2R_E_ARG, "marker %d (%g, %g) is outside the top face", m, mx, my);
    }
  }
  // tiles: Morton order of tet centroids, then greedy cuts at kTileTets tets / kTileVerts verts
  {
    std::vector<std::pair<uint32_t, int>> order(n_t);
    for (int e = 0; e < n_t; ++e) {
      uint32_t q[3];
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += X[3 * (size_t)tets[4 * (size_t)e + k] + a];
        s *= 0.25;
        const double u = (s - xlo[a]) / std::max(xhi[a] - xlo[a], 1e-300);
        q[a] = (uint32_t)std::min(1023.0, std::max(0.0, floor(u * 1024.0)));
      }
      order[e] = {spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2), e};
    }
    std::stable_sort(order.begin(), order.end());
    // tile boundaries: greedy cuts along the Morton order
    std::vector<int> bounds(1, 0);
    {
      std::unordered_map<int, int> seen;
      int cnt = 0;
      for (int i = 0; i < n_t; ++i) {
        const int e = order[i].second;
        int newv = 0;
        for (int k = 0; k < 4; ++k)
          if (!seen.count(tets[4 * (size_t)e + k])) ++newv;
        if (cnt == kTileTets || (int)seen.size() + newv > kTileVerts) {
          bounds.push_back(i);
          seen.clear();
          cnt = 0;
        }
        for (int k = 0; k < 4; ++k) seen.emplace(tets[4 * (size_t)e + k], 0);
        ++cnt;
      }
      bounds.push_back(n_t);
    }
    // inside each tile, deal tets into groups of 64 (one wavefront's lanes) so that
    // no vertex appears twice at the same tet-vertex slot within a group: the LDS
    // atomics of one instruction then never collide on an address
    {
      std::vector<std::pair<uint32_t, int>> reordered;
      reordered.reserve(n_t);
      for (size_t t = 0; t + 1 < bounds.size(); ++t) {
        const int b0 = bounds[t], b1 = bounds[t + 1];
        std::vector<int> rest;
        for (int i = b0; i < b1; ++i) rest.push_back(i);
        // fill each group of 64 in turn with the earliest tets that do not clash
        // with it; full groups keep every wavefront aligned with a group
        while (!rest.empty()) {
          std::array<std::vector<int>, 4> used;
          std::vector<int> take, keep;
          for (int i : rest) {
            const int e = order[i].second;
            bool ok = (int)take.size() < 64;
            for (int k = 0; k < 4 && ok; ++k) {
              const int v = tets[4 * (size_t)e + k];
              for (int u : used[k])
                if (u == v) { ok = false; break; }
            }
            if (ok) {
              take.push_back(i);
              for (int k = 0; k < 4; ++k) used[k].push_back(tets[4 * (size_t)e + k]);
            } else {
              keep.push_back(i);
            }
          }
          // not enough clash-free tets left: top the group up in order
          while ((int)take.size() < 64 && !keep.empty()) {
            take.push_back(keep.front());
            keep.erase(keep.begin());
          }
          for (int i : take) reordered.push_back(order[i]);
          rest.swap(keep);
        }
      }
      order.swap(reordered);
    }
    g.tet.resize(4 * (size_t)n_t);
    g.tet_local.resize(n_t);
    g.Dinv.resize(9 * (size_t)n_t);
    g.vol.resize(n_t);
    g.Dinv32.resize(9 * (size_t)n_t);
    g.vol32.resize(n_t);
    g.tile_tet.push_back(0);
    g.tile_vstart.push_back(0);
    std::unordered_map<int, int> local;
    std::vector<int> tile_v;
    int in_tile = 0;
    auto close_tile = [&](int next_e) {
      g.tile_tet.push_back(next_e);
      g.tile_verts.insert(g.tile_verts.end(), tile_v.begin(), tile_v.end());
      g.tile_vstart.push_back((int)g.tile_verts.size());
      local.clear();
      tile_v.clear();
      in_tile = 0;
    };
    size_t next_bound = 1;
    for (int i = 0; i < n_t; ++i) {
      const int e = order[i].second;
      if (i == bounds[next_bound] && i > 0) {
        close_tile(i);
        ++next_bound;
      }
      uint64_t loc = 0;
      for (int k = 0; k < 4; ++k) {
        const int v = tets[4 * (size_t)e + k];
        auto it = local.find(v);
        int l;
        if (it == local.end()) {
          l = (int)tile_v.size();
          local.emplace(v, l);
          tile_v.push_back(v);
        } else {
          l = it->second;
        }
        loc |= (uint64_t)l << (16 * k);
        g.tet[(size_t)k * n_t + i] = v;
      }
      g.tet_local[i] = loc;
      for (int k = 0; k < 9; ++k) {
        g.Dinv[(size_t)k * n_t + i] = Dinv[9 * (size_t)e + k];
        g.Dinv32[(size_t)k * n_t + i] = (float)Dinv[9 * (size_t)e + k];
      }
      g.vol[i] = vol[e];
      g.vol32[i] = (float)vol[e];
      ++in_tile;
    }
    close_tile(n_t);
    const int ntiles = (int)g.tile_tet.size() - 1;
    // number each tile's vertices in ascending global order, so that the
    // slot-parallel loads and stores of a tile's positions and sums touch as few
    // cache lines per wavefront as the mesh numbering allows
    for (int t = 0; t < ntiles; ++t) {
      const int e0 = g.tile_tet[t], e1 = g.tile_tet[t + 1];
      const int v0 = g.tile_vstart[t], nvt = g.tile_vstart[t + 1] - v0;
      std::vector<int> rank(nvt), nid(nvt);
      for (int l = 0; l < nvt; ++l) rank[l] = l;
      std::sort(rank.begin(), rank.end(),
                [&](int a, int b) { return g.tile_verts[v0 + a] < g.tile_verts[v0 + b]; });
      for (int r = 0; r < nvt; ++r) nid[rank[r]] = r;
      for (int i = e0; i < e1; ++i) {
        uint64_t loc = 0;
        for (int k = 0; k < 4; ++k)
          loc |= (uint64_t)nid[(int)((g.tet_local[i] >> (16 * k)) & 0xffff)] << (16 * k);
        g.tet_local[i] = loc;
      }
      std::vector<int> tv(nvt);
      for (int l = 0; l < nvt; ++l) tv[nid[l]] = g.tile_verts[v0 + l];
      std::copy(tv.begin(), tv.end(), g.tile_verts.begin() + v0);
    }
    std::vector<int> first(n_v, -1), last(n_v, -1);
    for (int t = 0; t < ntiles; ++t)
      for (int j = g.tile_vstart[t]; j < g.tile_vstart[t + 1]; ++j) {
        const int v = g.tile_verts[j];
        if (first[v] < 0) first[v] = t;
        last[v] = t;
      }
    g.tile_flags.resize(g.tile_verts.size());
    for (int t = 0; t < ntiles; ++t)
      for (int j = g.tile_vstart[t]; j < g.tile_vstart[t + 1]; ++j) {
        const int v = g.tile_verts[j];
        g.tile_flags[j] = (first[v] == t ? kFirstTouch : 0) | (last[v] == t ? kLastTouch : 0) |
                         (last[v] == t && g.fixed[v] ? kFixedLast : 0);
      }
  }
  c->gels.push_back(std::move(g));
  *gel_id = (int32_t)c->gels.size() - 1;
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_gel_info(const t2r_ctx* c, int32_t id, int32_t* out) {
  if (!c || !out || id < 0 || id >= (int)c->gels.size()) return T2R_E_ARG;
  const GelHost& g = c->gels[id];
  out[0] = g.n_v; out[1] = g.n_t; out[2] = g.n_sv; out[3] = g.n_se; out[4] = g.n_sf;
  out[5] = g.n_m; out[6] = (int)g.tile_tet.size() - 1; out[7] = g.n_top; out[8] = g.n_fixed;
  out[9] = pair_cap_of(c, g);
  return T2R_OK;
}

t2r_status t2r_gel_markers(const t2r_ctx* c, int32_t id, int32_t* tri, double* w) {
  if (!c || id < 0 || id >= (int)c->gels.size()) return T2R_E_ARG;
  const GelHost& g = c->gels[id];
  for (int m = 0; m < g.n_m; ++m)
    for (int k = 0; k < 3; ++k) {
      if (tri) tri[3 * m + k] = g.marker_tri[(size_t)k * g.n_m + m];
      if (w) w[3 * m + k] = g.marker_w[(size_t)k * g.n_m + m];
    }
  return T2R_OK;
}

t2r_status t2r_set_gel_markers(t2r_ctx* c, int32_t id, int32_t n_m, const int32_t* vertex,
                               const double* weight) {
  if (!c) return T2R_E_ARG;
  if (id < 0 || id >= (int)c->gels.size()) return fail(c, T2R_E_ARG, "bad gel id %d", id);
  if (c->committed) return fail(c, T2R_E_STATE, "markers can only change before the first GPU call");
  if (n_m < 0 || (n_m > 0 && (!vertex || !weight))) return fail(c, T2R_E_ARG, "bad marker arrays");
  GelHost& g = c->gels[id];
  for (int m = 0; m < n_m; ++m)
    for (int k = 0; k < 3; ++k) {
      const int v = vertex[3 * m + k];
      if (v < 0 || v >= g.n_v) return fail(c, T2R_E_ARG, "marker %d: vertex %d out of range", m, v);
      if (!isfinite(weight[3 * m + k])) return fail(c, T2R_E_ARG, "marker %d: weight not finite", m);
    }
  g.n_m = n_m;
  g.marker_tri.assign((size_t)3 * n_m, 0);
  g.marker_w.assign((size_t)3 * n_m, 0.0);
  for (int m = 0; m < n_m; ++m)
    for (int k = 0; k < 3; ++k) {
      g.marker_tri[(size_t)k * n_m + m] = vertex[3 * m + k];
      g.marker_w[(size_t)k * n_m + m] = weight[3 * m + k];
    }
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_add_indenter(t2r_ctx* c, int32_t n_v, const double* Y, int32_t n_f, const int32_t* tris,
                            int32_t* ind_id) {
  if (!c) return T2R_E_ARG;
  if (c->committed) return fail(c, T2R_E_STATE, "cannot add an indenter after the first GPU call");
  if (n_v < 3 || n_v > kMaxVerts || n_f < 1 || n_f > 2 * kMaxVerts) return fail(c, T2R_E_ARG, "bad indenter sizes");
  if (!Y || !tris || !ind_id) return fail(c, T2R_E_ARG, "null pointer");
  IndHost I;
  I.n_v = n_v;
  I.n_f = n_f;
  I.Y.resize(3 * (size_t)n_v);
  for (int a = 0; a < 3; ++a) { I.lo[a] = 1e300; I.hi[a] = -1e300; }
  for (int v = 0; v < n_v; ++v) {
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double y = Y[3 * (size_t)v + a];
      if (!isfinite(y)) return fail(c, T2R_E_ARG, "non-finite indenter vertex %d", v);
      I.Y[(size_t)a * n_v + v] = y;
      I.lo[a] = std::min(I.lo[a], y);
      I.hi[a] = std::max(I.hi[a], y);
      r2 += y * y;
    }
    I.r_max = std::max(I.r_max, sqrt(r2));
  }
  I.tri.resize(3 * (size_t)n_f);
  std::vector<std::pair<int, int>> es;
  for (int f = 0; f < n_f; ++f) {
    for (int k = 0; k < 3; ++k) {
      const int v = tris[3 * (size_t)f + k];
      if (v < 0 || v >= n_v) return fail(c, T2R_E_ARG, "indenter triangle %d has vertex id %d out of range", f, v);
      I.tri[(size_t)k * n_f + f] = v;
    }
    for (int k = 0; k < 3; ++k) {
      const int a = tris[3 * (size_t)f + k], b = tris[3 * (size_t)f + (k + 1) % 3];
      if (a == b) return fail(c, T2R_E_ARG, "indenter triangle %d is degenerate", f);
      es.push_back({std::min(a, b), std::max(a, b)});
    }
  }
  std::sort(es.begin(), es.end());
  es.erase(std::unique(es.begin(), es.end()), es.end());
  I.n_e = (int)es.size();
  I.edge.resize(2 * (size_t)I.n_e);
  for (int i = 0; i < I.n_e; ++i) { I.edge[i] = es[i].first; I.edge[I.n_e + i] = es[i].second; }
  // grids: cell ~ mean edge length, at most 64 cells per axis
  double mean_e = 0.0;
  for (int i = 0; i < I.n_e; ++i) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double d = Y[3 * (size_t)es[i].first + a] - Y[3 * (size_t)es[i].second + a];
      s += d * d;
    }
    mean_e += sqrt(s);
  }
  mean_e /= std::max(1, I.n_e);
  const double ext = std::max({I.hi[0] - I.lo[0], I.hi[1] - I.lo[1], I.hi[2] - I.lo[2]});
  // cells of about half the mean edge: a query then tests few primitives beyond
  // its own box; at most 96 cells per axis
  const double cell = std::max(0.5 * mean_e, ext / 96.0);
  auto box_of = [&](const int* ids, int k) {
    std::array<double, 6> b;
    for (int a = 0; a < 3; ++a) { b[a] = 1e300; b[3 + a] = -1e300; }
    for (int j = 0; j < k; ++j)
      for (int a = 0; a < 3; ++a) {
        const double y = Y[3 * (size_t)ids[j] + a];
        b[a] = std::min(b[a], y);
        b[3 + a] = std::max(b[3 + a], y);
      }
    return b;
  };
  std::vector<std::array<double, 6>> bv(n_v), be(I.n_e), bf(n_f);
  for (int v = 0; v < n_v; ++v) bv[v] = box_of(&v, 1);
  for (int i = 0; i < I.n_e; ++i) { int ids[2] = {es[i].first, es[i].second}; be[i] = box_of(ids, 2); }
  for (int f = 0; f < n_f; ++f) bf[f] = box_of(&tris[3 * (size_t)f], 3);
  build_grid(I.gv, bv, I.lo, I.hi, cell);
  build_grid(I.ge, be, I.lo, I.hi, cell);
  build_grid(I.gf, bf, I.lo, I.hi, cell);
  c->inds.push_back(std::move(I));
  *ind_id = (int32_t)c->inds.size() - 1;
  c->err.clear();
  return T2R_OK;
}

static bool valid_material(const t2r_material& m) {
  return m.E > 0 && m.nu > 0 && m.nu < 0.5 && m.mu_f >= 0 && m.eps_v > 0 && m.dhat > 0 && m.kappa > 0 &&
         isfinite(m.E) && isfinite(m.mu_f) && isfinite(m.eps_v) && isfinite(m.dhat) && isfinite(m.kappa);
}

static void material_to_dev(const t2r_material& m, EnvDev& d) {
  d.mu = m.E / (2.0 * (1.0 + m.nu));
  d.lam = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
  d.mu_f = m.mu_f;
  d.eps_v = m.eps_v;
  d.dhat = m.dhat;
  d.kappa = m.kappa;
}

t2r_status t2r_set_materials(t2r_ctx* c, int32_t n, const int32_t* env_ids, const t2r_material* mats) {
  if (!c) return T2R_E_ARG;
  if (n < 0 || (n > 0 && (!env_ids || !mats))) return fail(c, T2R_E_ARG, "bad arguments");
  for (int i = 0; i < n; ++i) {
    if (env_ids[i] < 0 || env_ids[i] >= (int)c->envs.size()) return fail(c, T2R_E_ARG, "bad env id %d", env_ids[i]);
    if (!valid_material(mats[i])) return fail(c, T2R_E_ARG, "env %d: invalid material", env_ids[i]);
  }
  if (c->committed) HIP_TRY(c, hipStreamSynchronize(c->stream));  // earlier work may read the descriptors
  ++c->layout_gen;
  for (int i = 0; i < n; ++i) {
    const int e = env_ids[i];
    c->envs[e].mat = mats[i];
    if (c->committed) {
      material_to_dev(mats[i], c->h_envs[e]);
      HIP_TRY(c, hipMemcpyAsync(c->d_envs + e, &c->h_envs[e], sizeof(EnvDev), hipMemcpyHostToDevice, c->stream));
      // list radii follow dhat: rebuild this env's lists on its next step
      HIP_TRY(c, hipMemsetAsync(c->d_lists + e, 0, sizeof(ListState), c->stream));
    }
  }
  if (c->committed) HIP_TRY(c, hipStreamSynchronize(c->stream));  // host copies are pageable
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_add_envs(t2r_ctx* c, int32_t n, const int32_t* gel_ids, const int32_t* ind_ids,
                        const t2r_material* mats, const double* pose0, int32_t* first_env) {
  if (!c) return T2R_E_ARG;
  if (c->committed) return fail(c, T2R_E_STATE, "cannot add environments after the first GPU call");
  if (n < 1 || !gel_ids || !ind_ids || !mats || !pose0) return fail(c, T2R_E_ARG, "bad arguments");
  std::vector<EnvHost> add;
  for (int i = 0; i < n; ++i) {
    EnvHost e;
    e.gel = gel_ids[i];
    e.ind = ind_ids[i];
    if (e.gel < 0 || e.gel >= (int)c->gels.size()) return fail(c, T2R_E_ARG, "env %d: bad gel id %d", i, e.gel);
    if (e.ind < 0 || e.ind >= (int)c->inds.size()) return fail(c, T2R_E_ARG, "env %d: bad indenter id %d", i, e.ind);
    const t2r_material& m = mats[i];
    if (!valid_material(m)) return fail(c, T2R_E_ARG, "env %d: invalid material", i);
    e.mat = m;
    double qn = 0.0;
    for (int k = 0; k < 7; ++k) {
      e.pose0[k] = pose0[7 * (size_t)i + k];
      if (!isfinite(e.pose0[k])) return fail(c, T2R_E_ARG, "env %d: non-finite pose", i);
      if (k >= 3) qn += e.pose0[k] * e.pose0[k];
    }
    if (!(qn > 0)) return fail(c, T2R_E_ARG, "env %d: zero quaternion", i);
    add.push_back(e);
  }
  if (first_env) *first_env = (int32_t)c->envs.size();
  c->envs.insert(c->envs.end(), add.begin(), add.end());
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_env_count(const t2r_ctx* c, int32_t* n_env, int64_t* total_verts) {
  if (!c) return T2R_E_ARG;
  if (n_env) *n_env = (int32_t)c->envs.size();
  if (total_verts) {
    int64_t s = 0;
    for (auto& e : c->envs) s += c->gels[e.gel].n_v;
    *total_verts = s;
  }
  return T2R_OK;
}

// Workgroup shape (one workgroup per env): automatic = 512 threads while the envs
// do not fill every compute unit at one workgroup each, else 256 (two per CU).
static int block_of(const t2r_ctx* c) {
  if (c->opts.block_size) return c->opts.block_size;
  return (int)c->envs.size() <= c->n_cu ? 512 : 256;
}

static StepParams step_params(t2r_ctx* c) {
  StepParams P{};
  P.gels = c->d_gels;
  P.inds = c->d_inds;
  P.envs = c->d_envs;
  P.n_env = (int)c->envs.size();
  P.x = c->d_x;
  P.xprev = c->d_xprev;
  P.g0 = c->d_g0;
  P.g1 = c->d_g1;
  P.diag = c->d_diag;
  P.p = c->d_p;
  P.pose_prev = c->d_pose_prev;
  P.pairs = c->d_pairs;
  P.pair_d = c->d_pair_d;
  P.outer = c->d_outer;
  P.lists = c->d_lists;
  P.xsnap = c->d_xsnap;
  P.fric = c->d_fric;
  P.vmap = c->d_vmap;
  P.imap = c->d_imap;
  P.islot_v = c->d_islot_v;
  P.oslot = c->d_oslot;
  P.pslot = c->d_pslot;
  P.slot_v = c->d_slot_v;
  P.stats = c->d_stats;
  P.order = nullptr;
  P.pose_lag = c->d_pose_lag;
  P.adj = c->d_adj;
  P.tape_x = nullptr;
  P.tape_q = nullptr;
  P.tape_stride = c->total_dofs;
  P.tape_k0 = 0;
  P.dL_du = nullptr;
  P.grad_out = nullptr;
  P.cg_tol = 1e-10;
  P.bw_steps = 0;
  P.bw_last = 0;
  P.n_steps = 1;
  P.markers_stride = 0;
  P.x_out_off = c->d_xout_off;
  P.clock_khz = c->clock_khz;
  P.tol = c->opts.tol;
  P.substep_tol = c->opts.substep_tol;
  P.max_iters = c->opts.max_iters;
  P.max_substeps = c->opts.max_substeps;
  P.max_evals = c->opts.max_evals;
  P.motion_mode = 0;
  P.motion_in = nullptr;
  P.motion_in2 = nullptr;
  P.motion_dt = 0.0;
  P.precision = c->opts.precision;
  P.ee_moll = c->opts.ee_mollifier;
  P.outer_mult = c->opts.outer_radius > 0.0 ? c->opts.outer_radius : 6.0;
  P.det = c->opts.deterministic;
  P.selfc = c->opts.self_contact;
  P.armijo = c->opts.armijo;
  P.warm_start = c->opts.warm_start;
  P.gap0 = c->d_gap;
  P.vel = c->d_vel;
  P.inertia_w = c->opts.dynamic ? c->opts.density / (c->opts.dt * c->opts.dt) : 0.0;
  P.dt = c->opts.dt;
  return P;
}

// One persistent launch of n_steps load steps; the targets come from poses
// (mode 0), velocities (1) or a relative motion (2); see StepParams.
static t2r_status launch_steps(t2r_ctx* c, int32_t n_steps, int mode, const double* in, const double* in2,
                               double dt, const int32_t* d_mask, double* d_markers, double* d_x,
                               int32_t* d_status) {
  if (!c) return T2R_E_ARG;
  if (!in || (mode == 2 && !in2)) return fail(c, T2R_E_ARG, "the step's input array is NULL");
  if (n_steps < 1) return fail(c, T2R_E_ARG, "n_steps must be >= 1 (got %d)", n_steps);
  if (mode == 1 && !(dt > 0.0 && isfinite(dt))) return fail(c, T2R_E_ARG, "dt must be positive and finite");
  if (c->envs.empty()) return fail(c, T2R_E_STATE, "no environments");
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  if (c->d_tape_x && c->tape_len + n_steps > c->tape_cap)
    return fail(c, T2R_E_STATE, "the tape holds %d more load steps (%d requested); t2r_record restarts it",
                c->tape_cap - c->tape_len, n_steps);
  StepParams P = step_params(c);
  P.n_steps = n_steps;
  if (c->d_tape_x) {
    P.tape_x = c->d_tape_x;
    P.tape_q = c->d_tape_q;
    P.tape_k0 = c->tape_len;
  }
  P.motion_mode = mode;
  if (mode == 0) {
    P.pose_in = in;
  } else {
    P.motion_in = in;
    P.motion_in2 = in2;
    P.motion_dt = dt;
  }
  P.env_mask = d_mask;
  P.markers_out = d_markers;
  P.markers_stride = 3 * c->total_markers;
  P.x_out = d_x;
  P.status_out = d_status;
  if (P.n_env > 1) {
    // longest previous launch first (see t2r_order_kernel)
    HIP_TRY(c, t2r_launch_order(&P, c->d_order, c->d_motion, c->stream));
    P.order = c->d_order;
  }
  HIP_TRY(c, t2r_launch_step(&P, block_of(c), c->stream));
  c->stepped = true;
  if (c->d_tape_x) c->tape_len += n_steps;
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_step_sequence(t2r_ctx* c, int32_t n_steps, const double* d_poses, const int32_t* d_mask,
                             double* d_markers, double* d_x, int32_t* d_status) {
  return launch_steps(c, n_steps, 0, d_poses, nullptr, 0.0, d_mask, d_markers, d_x, d_status);
}

t2r_status t2r_step_velocity(t2r_ctx* c, int32_t n_steps, double dt, const double* d_vel, const int32_t* d_mask,
                             double* d_markers, double* d_x, int32_t* d_status) {
  return launch_steps(c, n_steps, 1, d_vel, nullptr, dt, d_mask, d_markers, d_x, d_status);
}

t2r_status t2r_step_relative(t2r_ctx* c, int32_t n_steps, const double* d_rel0, const double* d_rel1,
                             const int32_t* d_mask, double* d_markers, double* d_x, int32_t* d_status) {
  return launch_steps(c, n_steps, 2, d_rel0, d_rel1, 0.0, d_mask, d_markers, d_x, d_status);
}

t2r_status t2r_set_pose_offsets(t2r_ctx* c, int32_t n, const int32_t* env_ids, const double* offsets) {
  if (!c) return T2R_E_ARG;
  if (n < 0 || (n > 0 && (!env_ids || !offsets))) return fail(c, T2R_E_ARG, "bad arguments");
  for (int i = 0; i < n; ++i) {
    if (env_ids[i] < 0 || env_ids[i] >= (int)c->envs.size()) return fail(c, T2R_E_ARG, "bad env id %d", env_ids[i]);
    for (int k = 0; k < 6; ++k)
      if (!isfinite(offsets[6 * (size_t)i + k])) return fail(c, T2R_E_ARG, "env %d: non-finite offset", env_ids[i]);
  }
  if (c->committed) HIP_TRY(c, hipStreamSynchronize(c->stream));  // earlier work may read the descriptors
  ++c->layout_gen;
  for (int i = 0; i < n; ++i) {
    EnvHost& e = c->envs[env_ids[i]];
    bool any = false;
    for (int k = 0; k < 6; ++k) {
      e.off[k] = offsets[6 * (size_t)i + k];
      any |= e.off[k] != 0.0;
    }
    e.has_off = any ? 1 : 0;
    if (c->committed) {
      EnvDev& d = c->h_envs[env_ids[i]];
      d.has_off = e.has_off;
      for (int k = 0; k < 6; ++k) d.off[k] = e.off[k];
      HIP_TRY(c, hipMemcpyAsync(c->d_envs + env_ids[i], &d, sizeof(EnvDev), hipMemcpyHostToDevice, c->stream));
    }
  }
  if (c->committed) HIP_TRY(c, hipStreamSynchronize(c->stream));  // host copies are pageable
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_set_densities(t2r_ctx* c, int32_t n, const int32_t* env_ids, const double* density) {
  if (!c) return T2R_E_ARG;
  if (n < 0 || (n > 0 && (!env_ids || !density))) return fail(c, T2R_E_ARG, "bad arguments");
  for (int i = 0; i < n; ++i) {
    if (env_ids[i] < 0 || env_ids[i] >= (int)c->envs.size()) return fail(c, T2R_E_ARG, "bad env id %d", env_ids[i]);
    if (!(density[i] >= 0.0) || !isfinite(density[i]))
      return fail(c, T2R_E_ARG, "env %d: density must be finite and >= 0", env_ids[i]);
  }
  if (c->committed) HIP_TRY(c, hipStreamSynchronize(c->stream));
  ++c->layout_gen;
  for (int i = 0; i < n; ++i) {
    c->envs[env_ids[i]].density = density[i];
    if (c->committed) {
      EnvDev& d = c->h_envs[env_ids[i]];
      d.density = density[i];
      HIP_TRY(c, hipMemcpyAsync(c->d_envs + env_ids[i], &d, sizeof(EnvDev), hipMemcpyHostToDevice, c->stream));
    }
  }
  if (c->committed) HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_set_gel_markers_knn(t2r_ctx* c, int32_t id, int32_t n_m, const double* markers_xy, int32_t k,
                                   double power) {
  if (!c) return T2R_E_ARG;
  if (id < 0 || id >= (int)c->gels.size()) return fail(c, T2R_E_ARG, "bad gel id %d", id);
  if (k < 1 || k > 3) return fail(c, T2R_E_ARG, "k must be 1, 2 or 3 (three nodes per marker), got %d", k);
  if (!(power > 0.0) || !isfinite(power)) return fail(c, T2R_E_ARG, "power must be positive");
  if (n_m < 0 || (n_m > 0 && !markers_xy)) return fail(c, T2R_E_ARG, "bad marker array");
  const GelHost& g = c->gels[id];
  if ((int)g.top_v.size() < k) return fail(c, T2R_E_ARG, "the top face has fewer than %d vertices", k);
  std::vector<int32_t> vert(3 * (size_t)n_m);
  std::vector<double> wt(3 * (size_t)n_m, 0.0);
  std::vector<std::pair<double, int>> dist(g.top_v.size());
  for (int m = 0; m < n_m; ++m) {
    const double mx = markers_xy[2 * (size_t)m], my = markers_xy[2 * (size_t)m + 1];
    if (!isfinite(mx) || !isfinite(my)) return fail(c, T2R_E_ARG, "non-finite marker %d", m);
    for (size_t j = 0; j < g.top_v.size(); ++j) {
      const int v = g.top_v[j];
      const double dx = g.X[v] - mx, dy = g.X[g.n_v + v] - my;
      dist[j] = {sqrt(dx * dx + dy * dy), v};
    }
    // the k nearest, ties by vertex id
    std::partial_sort(dist.begin(), dist.begin() + k, dist.end());
    for (int j = 0; j < 3; ++j) vert[3 * (size_t)m + j] = dist[0].second;
    if (dist[0].first <= 1e-12) {
      wt[3 * (size_t)m] = 1.0;  // a marker on a node takes that node alone
    } else {
      double sum = 0.0;
      for (int j = 0; j < k; ++j) {
        vert[3 * (size_t)m + j] = dist[j].second;
        wt[3 * (size_t)m + j] = 1.0 / pow(dist[j].first, power);
        sum += wt[3 * (size_t)m + j];
      }
      for (int j = 0; j < k; ++j) wt[3 * (size_t)m + j] /= sum;
    }
  }
  return t2r_set_gel_markers(c, id, n_m, vert.data(), wt.data());
}

t2r_status t2r_step(t2r_ctx* c, const double* d_pose, const int32_t* d_mask, double* d_markers, double* d_x,
                    int32_t* d_status) {
  return t2r_step_sequence(c, 1, d_pose, d_mask, d_markers, d_x, d_status);
}

t2r_status t2r_eval(t2r_ctx* c, int32_t env, const double* d_x, const double* d_p, const double* d_x_lag,
                    const double* pose, const double* pose_lag, double* d_grad, double* d_diag,
                    double* d_scalars) {
  if (!c) return T2R_E_ARG;
  if (env < 0 || env >= (int)c->envs.size()) return fail(c, T2R_E_ARG, "bad env id %d", env);
  if (!d_x || !pose || (d_x_lag && !pose_lag)) return fail(c, T2R_E_ARG, "null pointer");
  for (int k = 0; k < 7; ++k)
    if (!isfinite(pose[k]) || (pose_lag && d_x_lag && !isfinite(pose_lag[k])))
      return fail(c, T2R_E_ARG, "non-finite pose");
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  const EnvHost& E = c->envs[env];
  const GelHost& G = c->gels[E.gel];
  const int nv = G.n_v;
  EnvDev ed = c->h_envs[env];
  ed.voff = 0;
  ed.poff = 0;
  ed.foff = 0;
  ed.moff = 0;
  ed.ooff = 0;
  ed.snoff = 0;
  ed.vtxoff = 0;
  ed.imoff = 0;
  const int niv = c->inds[E.ind].n_v;
  // scratch (freed before returning)
  std::vector<void*> tmp;
  auto talloc = [&](size_t b) -> void* {
    void* p = nullptr;
    if (c->alloc) p = c->alloc(b, c->alloc_user);
    else if (hipMalloc(&p, b) != hipSuccess) p = nullptr;
    if (p) tmp.push_back(p);
    return p;
  };
  auto tfree = [&]() {
    (void)hipStreamSynchronize(c->stream);
    for (void* p : tmp) {
      if (c->free_fn) c->free_fn(p, c->alloc_user);
      else (void)hipFree(p);
    }
  };
  const size_t vb = 3 * (size_t)nv * sizeof(double);
  double* sx = (double*)talloc(vb);
  double* sxp = (double*)talloc(vb);
  double* sg0 = (double*)talloc(vb);
  double* sg1 = (double*)talloc(vb);
  double* sd = (double*)talloc(vb);
  double* sp = (double*)talloc(vb);
  int2* spairs = (int2*)talloc((size_t)ed.pair_cap * sizeof(int2));
  double* spd = (double*)talloc((size_t)ed.pair_cap * sizeof(double));
  int2* souter = (int2*)talloc((size_t)ed.outer_cap * sizeof(int2));
  ListState* slists = (ListState*)talloc(sizeof(ListState));
  double* ssnap = (double*)talloc(6 * (size_t)std::max(G.n_sv, 1) * sizeof(double));
  FricPair* sfric = (FricPair*)talloc((size_t)ed.fric_cap * sizeof(FricPair));
  EnvDev* senv = (EnvDev*)talloc(sizeof(EnvDev));
  double* sposes = (double*)talloc(14 * sizeof(double));
  EnvStats* sstats = (EnvStats*)talloc(sizeof(EnvStats));
  int* svmap = (int*)talloc((size_t)nv * sizeof(int));
  uint64_t* soslot = (uint64_t*)talloc((size_t)ed.outer_cap * sizeof(uint64_t));
  uint64_t* spslot = (uint64_t*)talloc((size_t)ed.pair_cap * sizeof(uint64_t));
  int* sslot_v = (int*)talloc((size_t)kGelSlots * sizeof(int));
  int* simap = (int*)talloc((size_t)niv * sizeof(int));
  int* sislot_v = (int*)talloc((size_t)kIndSlots * sizeof(int));
  if (tmp.size() != 21) { tfree(); return fail(c, T2R_E_NOMEM, "scratch allocation failed"); }
  double hp[14];
  for (int k = 0; k < 7; ++k) { hp[k] = pose[k]; hp[7 + k] = (pose_lag ? pose_lag[k] : pose[k]); }
  hipError_t he = hipSuccess;
  he = hipMemcpyAsync(senv, &ed, sizeof(EnvDev), hipMemcpyHostToDevice, c->stream);
  if (he == hipSuccess) he = hipMemcpyAsync(sposes, hp, sizeof hp, hipMemcpyHostToDevice, c->stream);
  if (he == hipSuccess) he = hipMemsetAsync(slists, 0, sizeof(ListState), c->stream);
  if (he == hipSuccess) he = hipMemsetAsync(svmap, 0, (size_t)nv * sizeof(int), c->stream);
  if (he == hipSuccess) he = hipMemsetAsync(simap, 0, (size_t)niv * sizeof(int), c->stream);
  if (he == hipSuccess) he = t2r_launch_aos_to_soa(d_x, sx, nv, c->stream);
  if (he == hipSuccess && d_p) he = t2r_launch_aos_to_soa(d_p, sp, nv, c->stream);
  if (he == hipSuccess && !d_p) he = hipMemsetAsync(sp, 0, vb, c->stream);
  if (he == hipSuccess && d_x_lag) he = t2r_launch_aos_to_soa(d_x_lag, sxp, nv, c->stream);
  if (he != hipSuccess) { tfree(); return fail(c, T2R_E_HIP, "eval setup: %s", hipGetErrorString(he)); }
  EvalParams Q{};
  Q.sp = step_params(c);
  Q.sp.inertia_w = 0.0;  // t2r_eval evaluates the quasi-static energy
  Q.sp.envs = senv;
  Q.sp.n_env = 1;
  Q.sp.x = sx;
  Q.sp.xprev = sxp;
  Q.sp.g0 = sg0;
  Q.sp.g1 = sg1;
  Q.sp.diag = sd;
  Q.sp.p = sp;
  Q.sp.pairs = spairs;
  Q.sp.pair_d = spd;
  Q.sp.outer = souter;
  Q.sp.lists = slists;
  Q.sp.xsnap = ssnap;
  Q.sp.fric = sfric;
  Q.sp.vmap = svmap;
  Q.sp.oslot = soslot;
  Q.sp.pslot = spslot;
  Q.sp.slot_v = sslot_v;
  Q.sp.imap = simap;
  Q.sp.islot_v = sislot_v;
  Q.sp.stats = sstats;
  Q.env = 0;
  Q.pose = sposes;
  Q.pose_lag = sposes + 7;
  Q.has_lag = d_x_lag ? 1 : 0;
  Q.has_p = d_p ? 1 : 0;
  Q.grad_out = d_grad;
  Q.diag_out = d_diag;
  Q.scalars_out = d_scalars;
  he = t2r_launch_eval(&Q, 256, c->stream);
  int32_t est = 0;
  if (he == hipSuccess) he = hipMemcpyAsync(&est, &sstats->status, sizeof est, hipMemcpyDeviceToHost, c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  tfree();
  if (he != hipSuccess) return fail(c, T2R_E_HIP, "eval: %s", hipGetErrorString(he));
  if (est & T2R_ENV_PAIR_OVERFLOW)
    return fail(c, T2R_E_NOMEM, "contact pair list capacity %d exceeded (raise it with t2r_set_pair_capacity)",
                ed.pair_cap);
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_get_stats(t2r_ctx* c, void* out, size_t bytes) {
  if (!c || !out) return T2R_E_ARG;
  if (!c->committed) return fail(c, T2R_E_STATE, "no step has run");
  const size_t need = c->envs.size() * sizeof(t2r_env_stats);
  if (bytes < need) return fail(c, T2R_E_ARG, "buffer too small: %zu < %zu", bytes, need);
  static_assert(sizeof(t2r_env_stats) == sizeof(EnvStats), "stats layout");
  HIP_TRY(c, hipMemcpyAsync(out, c->d_stats, need, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_state_size(const t2r_ctx* c, int64_t* n) {
  if (!c || !n) return T2R_E_ARG;
  int64_t s = 0;
  for (auto& e : c->envs) s += 3 * (int64_t)c->gels[e.gel].n_v + 7;
  *n = s;
  return T2R_OK;
}

t2r_status t2r_get_state(t2r_ctx* c, double* d_state) {
  if (!c || !d_state) return T2R_E_ARG;
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  StepParams P = step_params(c);
  HIP_TRY(c, t2r_launch_pack_state(&P, nullptr, d_state, c->d_state_off, 1, c->stream));
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_set_state(t2r_ctx* c, const double* d_state) {
  if (!c || !d_state) return T2R_E_ARG;
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  StepParams P = step_params(c);
  HIP_TRY(c, t2r_launch_pack_state(&P, d_state, nullptr, c->d_state_off, 0, c->stream));
  // positions changed arbitrarily: every neighbour list must be rebuilt
  HIP_TRY(c, hipMemsetAsync(c->d_lists, 0, c->envs.size() * sizeof(ListState), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_gap, 0, c->envs.size() * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_vel, 0, (size_t)c->total_dofs * sizeof(double), c->stream));
  s = tape_seed(c);
  if (s != T2R_OK) return s;
  c->err.clear();
  return T2R_OK;
}

// Checkpoint: positions x_s, x_{s-1}, velocities, poses q_s and q_{s-1} and the
// warm start's starting distance, each as the whole array in device order.
t2r_status t2r_checkpoint_size(const t2r_ctx* c, int64_t* n) {
  if (!c || !n) return T2R_E_ARG;
  int64_t dofs = 0;
  for (auto& e : c->envs) dofs += 3 * (int64_t)c->gels[e.gel].n_v;
  *n = 3 * dofs + 15 * (int64_t)c->envs.size();
  return T2R_OK;
}

// The checkpoint's arrays in order: {device array, doubles}.
static void checkpoint_parts(t2r_ctx* c, double* parts[6], size_t n[6]) {
  const size_t dofs = (size_t)c->total_dofs, ne = c->envs.size();
  parts[0] = c->d_x; n[0] = dofs;
  parts[1] = c->d_xprev; n[1] = dofs;
  parts[2] = c->d_vel; n[2] = dofs;
  parts[3] = c->d_pose_prev; n[3] = 7 * ne;
  parts[4] = c->d_pose_lag; n[4] = 7 * ne;
  parts[5] = c->d_gap; n[5] = ne;
}

t2r_status t2r_save_checkpoint(t2r_ctx* c, double* d_buf) {
  if (!c || !d_buf) return T2R_E_ARG;
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  double* parts[6];
  size_t n[6], off = 0;
  checkpoint_parts(c, parts, n);
  for (int k = 0; k < 6; ++k) {
    HIP_TRY(c, hipMemcpyAsync(d_buf + off, parts[k], n[k] * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    off += n[k];
  }
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_load_checkpoint(t2r_ctx* c, const double* d_buf) {
  if (!c || !d_buf) return T2R_E_ARG;
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  double* parts[6];
  size_t n[6], off = 0;
  checkpoint_parts(c, parts, n);
  for (int k = 0; k < 6; ++k) {
    HIP_TRY(c, hipMemcpyAsync(parts[k], d_buf + off, n[k] * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    off += n[k];
  }
  // neighbour lists are not part of a checkpoint: rebuilt at the next step
  HIP_TRY(c, hipMemsetAsync(c->d_lists, 0, c->envs.size() * sizeof(ListState), c->stream));
  s = tape_seed(c);
  if (s != T2R_OK) return s;
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_reset_envs(t2r_ctx* c, const int32_t* ids, int32_t n) {
  if (!c || (n > 0 && !ids) || n < 0) return T2R_E_ARG;
  for (int i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= (int)c->envs.size()) return fail(c, T2R_E_ARG, "bad env id %d", ids[i]);
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  for (int i = 0; i < n; ++i) {
    const EnvHost& e = c->envs[ids[i]];
    const GelHost& g = c->gels[e.gel];
    const EnvDev& ed = c->h_envs[ids[i]];
    HIP_TRY(c, hipMemcpyAsync(c->d_x + ed.voff, g.dev.X, 3 * (size_t)g.n_v * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    double q0[7];
    start_pose(e, q0);
    HIP_TRY(c, hipMemcpyAsync(c->d_pose_prev + 7 * (size_t)ids[i], q0, 7 * sizeof(double),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_pose_lag + 7 * (size_t)ids[i], q0, 7 * sizeof(double),
                              hipMemcpyHostToDevice, c->stream));  // no motion history
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // q0 is a pageable stack copy
    HIP_TRY(c, hipMemsetAsync(c->d_lists + ids[i], 0, sizeof(ListState), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_gap + ids[i], 0, sizeof(double), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_vel + ed.voff, 0, 3 * (size_t)g.n_v * sizeof(double), c->stream));
  }
  s = tape_seed(c);
  if (s != T2R_OK) return s;
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // host pose0 copies are pageable
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_set_pair_capacity(t2r_ctx* c, int32_t cap) {
  if (!c || cap < 0) return T2R_E_ARG;
  if (cap > (1 << 24)) return fail(c, T2R_E_ARG, "pair capacity too large");
  const int32_t old = c->opts.pair_capacity;
  c->opts.pair_capacity = cap;
  ++c->layout_gen;
  if (c->committed && cap != old) {
    const t2r_status s = relayout_lists(c);
    if (s != T2R_OK) { c->opts.pair_capacity = old; return s; }
  }
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_get_opts(const t2r_ctx* c, t2r_solver_opts* out) {
  if (!c || !out) return T2R_E_ARG;
  *out = c->opts;
  return T2R_OK;
}

t2r_status t2r_set_opts(t2r_ctx* c, const t2r_solver_opts* o) {
  if (!c || !o) return T2R_E_ARG;
  t2r_status s = check_opts(c, o);
  if (s != T2R_OK) return s;
  if (o->pair_capacity != c->opts.pair_capacity) {
    s = t2r_set_pair_capacity(c, o->pair_capacity);
    if (s != T2R_OK) return s;
  }
  c->opts = *o;
  ++c->layout_gen;
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_layout_generation(const t2r_ctx* c, int64_t* gen) {
  if (!c || !gen) return T2R_E_ARG;
  *gen = c->layout_gen;
  return T2R_OK;
}

t2r_status t2r_record(t2r_ctx* c, int32_t max_steps) {
  if (!c || max_steps < 0) return T2R_E_ARG;
  if (c->envs.empty()) return fail(c, T2R_E_STATE, "no environments");
  t2r_status s = commit(c);
  if (s != T2R_OK) return s;
  if (c->d_tape_x) HIP_TRY(c, hipStreamSynchronize(c->stream));
  dev_free(c, c->d_tape_x);
  dev_free(c, c->d_tape_q);
  c->d_tape_x = c->d_tape_q = nullptr;
  c->tape_cap = c->tape_len = 0;
  ++c->layout_gen;
  if (max_steps == 0) {
    c->err.clear();
    return T2R_OK;
  }
  const size_t entries = (size_t)max_steps + 1;
  c->d_tape_x = alloc_n<double>(c, entries * (size_t)c->total_dofs);
  c->d_tape_q = alloc_n<double>(c, entries * 7 * c->envs.size());
  if (!c->d_tape_x || !c->d_tape_q) {
    dev_free(c, c->d_tape_x);
    dev_free(c, c->d_tape_q);
    c->d_tape_x = c->d_tape_q = nullptr;
    return fail(c, T2R_E_NOMEM, "tape of %d load steps does not fit", max_steps);
  }
  c->tape_cap = max_steps;
  s = tape_seed(c);
  if (s != T2R_OK) return s;
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_tape_read(t2r_ctx* c, int32_t entry, double* d_state) {
  if (!c || !d_state) return T2R_E_ARG;
  if (!c->d_tape_x) return fail(c, T2R_E_STATE, "no tape: call t2r_record before the load steps");
  if (entry < 0 || entry > c->tape_len)
    return fail(c, T2R_E_ARG, "entry must be in [0, %d], got %d", c->tape_len, entry);
  StepParams P = step_params(c);
  P.x = c->d_tape_x + (size_t)entry * (size_t)c->total_dofs;
  P.pose_prev = c->d_tape_q + (size_t)entry * 7 * c->envs.size();
  HIP_TRY(c, t2r_launch_pack_state(&P, nullptr, d_state, c->d_state_off, 1, c->stream));
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_tape_length(const t2r_ctx* c, int32_t* n_steps) {
  if (!c || !n_steps) return T2R_E_ARG;
  *n_steps = c->d_tape_x ? c->tape_len : -1;
  return T2R_OK;
}

static t2r_status launch_adjoint(t2r_ctx* c, StepParams& P, const double* d_dL_du, double* d_grad) {
  if (c->opts.dynamic) return fail(c, T2R_E_UNSUPPORTED, "the adjoint covers the quasi-static form (dynamic = 0)");
  P.dL_du = d_dL_du;
  P.grad_out = d_grad;
  P.markers_stride = 3 * c->total_markers;
  HIP_TRY(c, t2r_launch_backward(&P, block_of(c), c->stream));
  c->err.clear();
  return T2R_OK;
}

t2r_status t2r_backward_sequence(t2r_ctx* c, int32_t n_steps, const double* d_dL_du, double* d_grad) {
  if (!c) return T2R_E_ARG;
  if (!d_dL_du || !d_grad) return fail(c, T2R_E_ARG, "d_dL_du and d_grad are required");
  if (!c->d_tape_x) return fail(c, T2R_E_STATE, "no tape: call t2r_record before the load steps");
  if (n_steps < 1 || n_steps > c->tape_len)
    return fail(c, T2R_E_ARG, "n_steps must be in [1, %d] (the recorded load steps), got %d", c->tape_len,
                n_steps);
  StepParams P = step_params(c);
  P.tape_x = c->d_tape_x;
  P.tape_q = c->d_tape_q;
  P.bw_steps = n_steps;
  P.bw_last = c->tape_len;
  return launch_adjoint(c, P, d_dL_du, d_grad);
}

t2r_status t2r_backward(t2r_ctx* c, const double* d_dL_du, double* d_grad) {
  if (!c) return T2R_E_ARG;
  for (size_t i = 0; i < c->envs.size(); ++i)
    if (c->envs[i].mat.mu_f != 0.0)
      return fail(c, T2R_E_UNSUPPORTED,
                  "env %zu has mu_f = %g: with friction the equilibrium depends on the earlier steps "
                  "(t2r_record + t2r_backward_sequence)", i, c->envs[i].mat.mu_f);
  if (!d_dL_du || !d_grad) return fail(c, T2R_E_ARG, "d_dL_du and d_grad are required");
  if (!c->committed || !c->stepped) return fail(c, T2R_E_STATE, "no load step has run");
  // a two-entry tape: (x_{s-1}, q_{s-1}) and (x_s, q_s) of the last load step
  const size_t nd = (size_t)c->total_dofs, nq = 7 * c->envs.size();
  if (!c->d_bw_x) {
    c->d_bw_x = alloc_n<double>(c, 2 * nd);
    c->d_bw_q = alloc_n<double>(c, 2 * nq);
    if (!c->d_bw_x || !c->d_bw_q) {
      dev_free(c, c->d_bw_x);
      dev_free(c, c->d_bw_q);
      c->d_bw_x = c->d_bw_q = nullptr;
      return fail(c, T2R_E_NOMEM, "adjoint scratch");
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_bw_x, c->d_xprev, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_bw_x + nd, c->d_x, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_bw_q, c->d_pose_lag, nq * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_bw_q + nq, c->d_pose_prev, nq * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
  StepParams P = step_params(c);
  P.tape_x = c->d_bw_x;
  P.tape_q = c->d_bw_q;
  P.bw_steps = 1;
  P.bw_last = 1;
  return launch_adjoint(c, P, d_dL_du, d_grad);
}

t2r_status t2r_backward_static(t2r_ctx* c, const double* d_dL_du, double* d_grad) {
  if (!c) return T2R_E_ARG;
  if (!d_dL_du || !d_grad) return fail(c, T2R_E_ARG, "d_dL_du and d_grad are required");
  // sizes first: a context whose two-entry tape does not fit is refused before any GPU use
  size_t nd = 0;  // 3 x the vertices of every env (the context may not have uploaded yet)
  for (const EnvHost& e : c->envs) nd += 3 * (size_t)c->gels[e.gel].n_v;
  const size_t nq = 7 * c->envs.size();
  const size_t need = 2 * nd + 2 * nq, cap = t2r_static_scratch_capacity();
  if (need > cap)
    return fail(c, T2R_E_ARG,
                "t2r_backward_static: the adjoint tape needs %zu doubles (2 x (3 x %zu vertices + 7 x %zu envs)) "
                "and the static workspace holds %zu; use t2r_backward", need, nd / 3, c->envs.size(), cap);
  for (size_t i = 0; i < c->envs.size(); ++i)
    if (c->envs[i].mat.mu_f != 0.0)
      return fail(c, T2R_E_UNSUPPORTED, "env %zu has mu_f = %g (t2r_record + t2r_backward_sequence)", i,
                  c->envs[i].mat.mu_f);
  if (!c->committed || !c->stepped) return fail(c, T2R_E_STATE, "no load step has run");
  if (c->opts.dynamic) return fail(c, T2R_E_UNSUPPORTED, "the adjoint covers the quasi-static form (dynamic = 0)");
  int cur = -1;
  HIP_TRY(c, hipGetDevice(&cur));
  if (cur != c->device) HIP_TRY(c, hipSetDevice(c->device));
  double* ws = nullptr;
  size_t n = 0;
  const hipError_t e = t2r_static_scratch(c->device, &ws, &n);
  if (cur != c->device) HIP_TRY(c, hipSetDevice(cur));
  if (e != hipSuccess) return fail(c, T2R_E_HIP, "static workspace: %s", hipGetErrorString(e));
  double* tx = ws;
  double* tq = ws + 2 * nd;
  HIP_TRY(c, hipMemcpyAsync(tx, c->d_xprev, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(tx + nd, c->d_x, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(tq, c->d_pose_lag, nq * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(tq + nq, c->d_pose_prev, nq * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  StepParams P = step_params(c);
  P.tape_x = tx;
  P.tape_q = tq;
  P.bw_steps = 1;
  P.bw_last = 1;
  return launch_adjoint(c, P, d_dL_du, d_grad);
}

}  // extern "C"

// ===========================================================================
namespace {

t2r_status upload_gel(t2r_ctx* c, GelHost& g) {
  GelDev& d = g.dev;
  d.n_v = g.n_v; d.n_t = g.n_t; d.n_tiles = (int)g.tile_tet.size() - 1;
  d.n_sv = g.n_sv; d.n_se = g.n_se; d.n_sf = g.n_sf; d.n_m = g.n_m;
  d.vol_total = g.vol_total;
  d.diag_rest_max = g.diag_rest_max;
  t2r_status s;
#define UP(field, vec) if ((s = upload(c, vec, &d.field)) != T2R_OK) return s
  UP(X, g.X); UP(fixed, g.fixed); UP(tet, g.tet); UP(tet_local, g.tet_local); UP(Dinv, g.Dinv);
  UP(vol, g.vol); UP(Dinv32, g.Dinv32); UP(vol32, g.vol32); UP(tile_tet, g.tile_tet);
  UP(tile_vstart, g.tile_vstart); UP(tile_verts, g.tile_verts); UP(tile_flags, g.tile_flags);
  UP(surf_v, g.surf_v); UP(surf_e, g.surf_e); UP(surf_f, g.surf_f); UP(marker_tri, g.marker_tri);
  UP(marker_w, g.marker_w);
  {
    std::vector<double> vm(g.n_v, 0.0);
    for (int e = 0; e < g.n_t; ++e)
      for (int k = 0; k < 4; ++k) vm[g.tet[k * g.n_t + e]] += 0.25 * g.vol[e];
    UP(vmass, vm);
  }
#undef UP
  return T2R_OK;
}

t2r_status upload_grid(t2r_ctx* c, IndHost::GridHost& h, Grid& d) {
  for (int a = 0; a < 3; ++a) { d.origin[a] = h.origin[a]; d.dims[a] = h.dims[a]; }
  d.inv_cell = h.inv_cell;
  d.n_prim = h.n;
  t2r_status s;
  if ((s = upload(c, h.start, &d.start)) != T2R_OK) return s;
  if ((s = upload(c, h.items, &d.items)) != T2R_OK) return s;
  return upload(c, h.box, &d.box);
}

t2r_status upload_ind(t2r_ctx* c, IndHost& I) {
  IndDev& d = I.dev;
  d.n_v = I.n_v; d.n_f = I.n_f; d.n_e = I.n_e; d.r_max = I.r_max;
  for (int a = 0; a < 3; ++a) { d.box_lo[a] = I.lo[a]; d.box_hi[a] = I.hi[a]; }
  t2r_status s;
  if ((s = upload(c, I.Y, &d.Y)) != T2R_OK) return s;
  if ((s = upload(c, I.tri, &d.tri)) != T2R_OK) return s;
  if ((s = upload(c, I.edge, &d.edge)) != T2R_OK) return s;
  if ((s = upload_grid(c, I.gv, d.gv)) != T2R_OK) return s;
  if ((s = upload_grid(c, I.ge, d.ge)) != T2R_OK) return s;
  return upload_grid(c, I.gf, d.gf);
}

template <typename T>
T* alloc_n(t2r_ctx* c, size_t n) {
  return (T*)dev_alloc(c, n * sizeof(T));
}

int pair_cap_of(const t2r_ctx* c, const GelHost& g) {
  const int cap = c->opts.pair_capacity;
  return cap > 0 ? cap : std::max(8192, 3 * (g.n_sv + g.n_se + g.n_sf));
}

// After the first GPU call: new pair-list capacities. The lists are rebuilt on
// the next step anyway, so the old buffers are dropped (state vectors kept)
// and every env's lists are marked invalid.
t2r_status relayout_lists(t2r_ctx* c) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  ++c->layout_gen;
  std::vector<EnvDev> he = c->h_envs;
  long long poff = 0, foff = 0, ooff = 0;
  for (size_t i = 0; i < he.size(); ++i) {
    EnvDev& d = he[i];
    const int cap = pair_cap_of(c, c->gels[d.gel]);
    d.pair_cap = cap;
    d.fric_cap = std::max(1024, cap / 2);
    d.outer_cap = 4 * cap;
    d.poff = poff;
    d.foff = foff;
    d.ooff = ooff;
    poff += cap;
    foff += d.fric_cap;
    ooff += d.outer_cap;
  }
  int2* pairs = alloc_n<int2>(c, (size_t)poff);
  double* pair_d = alloc_n<double>(c, (size_t)poff);
  int2* outer = alloc_n<int2>(c, (size_t)ooff);
  uint64_t* oslot = alloc_n<uint64_t>(c, (size_t)ooff);
  uint64_t* pslot = alloc_n<uint64_t>(c, (size_t)poff);
  FricPair* fric = alloc_n<FricPair>(c, (size_t)foff);
  const EnvDev* de = nullptr;
  t2r_status s = T2R_OK;
  if (pairs && pair_d && outer && oslot && pslot && fric) s = upload(c, he, &de);
  if (!(pairs && pair_d && outer && oslot && pslot && fric) || s != T2R_OK || !de) {
    for (void* p : {(void*)pairs, (void*)pair_d, (void*)outer, (void*)oslot, (void*)pslot, (void*)fric})
      dev_free(c, p);
    return fail(c, T2R_E_NOMEM, "pair list allocation failed (%lld inner pairs)", poff);
  }
  for (void* p : {(void*)c->d_pairs, (void*)c->d_pair_d, (void*)c->d_outer, (void*)c->d_oslot,
                  (void*)c->d_pslot, (void*)c->d_fric, (void*)c->d_envs})
    dev_free(c, p);
  c->d_pairs = pairs;
  c->d_pair_d = pair_d;
  c->d_outer = outer;
  c->d_oslot = oslot;
  c->d_pslot = pslot;
  c->d_fric = fric;
  c->d_envs = (EnvDev*)de;
  c->h_envs = he;
  HIP_TRY(c, hipMemsetAsync(c->d_lists, 0, c->envs.size() * sizeof(ListState), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return T2R_OK;
}

t2r_status commit(t2r_ctx* c) {
  if (c->committed) return T2R_OK;
  ++c->layout_gen;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count == 0)
    return fail(c, T2R_E_HIP, "no HIP device available");
  {
    int dev = 0, khz = 0;
    HIP_TRY(c, hipGetDevice(&dev));
    c->device = dev;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      c->clock_khz = (double)khz;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      c->n_cu = cu;
  }
  t2r_status s;
  for (auto& g : c->gels)
    if ((s = upload_gel(c, g)) != T2R_OK) { dev_free_all(c); return s; }
  for (auto& I : c->inds)
    if ((s = upload_ind(c, I)) != T2R_OK) { dev_free_all(c); return s; }
  std::vector<GelDev> hg;
  for (auto& g : c->gels) hg.push_back(g.dev);
  std::vector<IndDev> hi;
  for (auto& I : c->inds) hi.push_back(I.dev);
  const GelDev* dg;
  const IndDev* di;
  if ((s = upload(c, hg, &dg)) != T2R_OK) { dev_free_all(c); return s; }
  if ((s = upload(c, hi, &di)) != T2R_OK) { dev_free_all(c); return s; }
  c->d_gels = (GelDev*)dg;
  c->d_inds = (IndDev*)di;
  // per-env layout
  c->h_envs.clear();
  long long voff = 0, poff = 0, foff = 0, moff = 0, vtot = 0, soff = 0, ooff = 0, snoff = 0, imtot = 0;
  std::vector<long long> xoff, sofs;
  for (auto& e : c->envs) {
    const GelHost& g = c->gels[e.gel];
    EnvDev d{};
    d.gel = e.gel;
    d.ind = e.ind;
    material_to_dev(e.mat, d);
    d.has_off = e.has_off;
    for (int k = 0; k < 6; ++k) d.off[k] = e.off[k];
    d.density = e.density;
    const int cap = pair_cap_of(c, g);
    d.pair_cap = cap;
    d.fric_cap = std::max(1024, cap / 2);
    d.outer_cap = 4 * cap;
    d.ooff = ooff;
    d.snoff = snoff;
    d.vtxoff = vtot;
    d.imoff = imtot;
    d.voff = voff;
    d.poff = poff;
    d.foff = foff;
    d.moff = moff;
    xoff.push_back(vtot);
    sofs.push_back(soff);
    voff += 3 * (long long)g.n_v;
    poff += cap;
    foff += d.fric_cap;
    ooff += d.outer_cap;
    snoff += 6 * (long long)g.n_sv;
    moff += g.n_m;
    vtot += g.n_v;
    imtot += c->inds[e.ind].n_v;
    soff += 3 * (long long)g.n_v + 7;
    c->h_envs.push_back(d);
  }
  c->total_dofs = voff;
  c->total_verts = vtot;
  c->total_markers = moff;
  c->state_size = soff;
  const GelDev* dummy;
  (void)dummy;
  const EnvDev* de;
  if ((s = upload(c, c->h_envs, &de)) != T2R_OK) { dev_free_all(c); return s; }
  c->d_envs = (EnvDev*)de;
  const long long* dx;
  if ((s = upload(c, xoff, &dx)) != T2R_OK) { dev_free_all(c); return s; }
  c->d_xout_off = (long long*)dx;
  if ((s = upload(c, sofs, &dx)) != T2R_OK) { dev_free_all(c); return s; }
  c->d_state_off = (long long*)dx;
  const size_t nd = (size_t)voff;
  c->d_x = alloc_n<double>(c, nd);
  c->d_xprev = alloc_n<double>(c, nd);
  c->d_g0 = alloc_n<double>(c, nd);
  c->d_g1 = alloc_n<double>(c, nd);
  c->d_diag = alloc_n<double>(c, nd);
  c->d_p = alloc_n<double>(c, nd);
  c->d_pose_prev = alloc_n<double>(c, 7 * c->envs.size());
  c->d_pairs = alloc_n<int2>(c, (size_t)poff);
  c->d_pair_d = alloc_n<double>(c, (size_t)poff);
  c->d_outer = alloc_n<int2>(c, (size_t)ooff);
  c->d_lists = alloc_n<ListState>(c, c->envs.size());
  c->d_xsnap = alloc_n<double>(c, (size_t)std::max(snoff, 1LL));
  c->d_fric = alloc_n<FricPair>(c, (size_t)foff);
  c->d_vmap = alloc_n<int>(c, (size_t)vtot);
  c->d_oslot = alloc_n<uint64_t>(c, (size_t)ooff);
  c->d_pslot = alloc_n<uint64_t>(c, (size_t)poff);
  c->d_slot_v = alloc_n<int>(c, c->envs.size() * (size_t)kGelSlots);
  c->d_imap = alloc_n<int>(c, (size_t)std::max(imtot, 1LL));
  c->d_islot_v = alloc_n<int>(c, c->envs.size() * (size_t)kIndSlots);
  c->d_stats = alloc_n<EnvStats>(c, c->envs.size());
  c->d_order = alloc_n<int>(c, c->envs.size());
  c->d_motion = alloc_n<double>(c, c->envs.size());
  c->d_pose_lag = alloc_n<double>(c, 7 * c->envs.size());
  c->d_adj = alloc_n<double>(c, nd);
  c->d_gap = alloc_n<double>(c, c->envs.size());
  c->d_vel = alloc_n<double>(c, nd);
  if (!c->d_vel || !c->d_gap || !c->d_x || !c->d_xprev || !c->d_g0 || !c->d_g1 || !c->d_diag || !c->d_p || !c->d_pose_prev ||
      !c->d_pairs || !c->d_pair_d || !c->d_outer || !c->d_lists || !c->d_xsnap || !c->d_fric ||
      !c->d_vmap || !c->d_oslot || !c->d_pslot || !c->d_slot_v || !c->d_imap || !c->d_islot_v ||
      !c->d_stats || !c->d_order || !c->d_motion || !c->d_pose_lag || !c->d_adj) {
    dev_free_all(c);
    return fail(c, T2R_E_NOMEM, "state allocation failed (%lld DOFs)", voff);
  }
  // initial state: x = X, p = 0, pose_prev = pose0
  std::vector<double> pose(7 * c->envs.size());
  for (size_t i = 0; i < c->envs.size(); ++i) {
    const GelHost& g = c->gels[c->envs[i].gel];
    HIP_TRY(c, hipMemcpyAsync(c->d_x + c->h_envs[i].voff, g.dev.X, 3 * (size_t)g.n_v * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    start_pose(c->envs[i], &pose[7 * i]);
  }
  HIP_TRY(c, hipMemsetAsync(c->d_p, 0, nd * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_stats, 0, c->envs.size() * sizeof(EnvStats), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_motion, 0, c->envs.size() * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_gap, 0, c->envs.size() * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_vel, 0, nd * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_lists, 0, c->envs.size() * sizeof(ListState), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_vmap, 0, (size_t)vtot * sizeof(int), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_imap, 0, (size_t)std::max(imtot, 1LL) * sizeof(int), c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_pose_prev, pose.data(), pose.size() * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_pose_lag, pose.data(), pose.size() * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // host staging vectors go out of scope
  c->committed = true;
  return T2R_OK;
}

}  // namespace
