// C ABI of libdgrtm: host driver of the multi-rate DG solver and the RTM procedure.
#include "../../include/dgrtm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "setup.hpp"

using namespace dgrtm;

namespace {
thread_local std::string g_err;

dgrtm_status fail(dgrtm_status code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(DGRTM_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// bump allocator inside a caller-provided device workspace (256-byte aligned slices)
struct Bump {
  char *base = nullptr;
  size_t used = 0, cap = 0;
  template <class T>
  T *take(size_t n) {
    used = (used + 255) / 256 * 256;
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used += n * sizeof(T);
    return p;
  }
};
}  // namespace

int32_t dgrtm::report_error(int32_t code, const std::string &msg) { return fail(code, msg); }

struct dgrtm_mesh_s {
  RefOps ref;
  HostMesh hm;
  bool bound = false;
  hipStream_t stream = nullptr;
  // device
  float *geo = nullptr;
  int *nbr = nullptr, *ncode = nullptr, *eflag = nullptr;
  float *ops = nullptr;
  uint32_t *ops_bf16 = nullptr;
  int8_t *nbr_index = nullptr;
  int64_t *s2u = nullptr;
  uint32_t *tile_ctr = nullptr;  // per shot slot: next-tile and finished-wave counters of the step kernel
  int64_t max_groups = 0;        // cap on step-launch work-groups (0: one per compute unit)
  std::vector<int> h_eflag;  // base flags (valid, has finer neighbour)
  // boundary faces (for the boundary-trace record): sorted position * 4 + face, finest level first
  int *bface = nullptr;
  int64_t n_bfaces = 0;
  int64_t bnd_cnt[kMaxLevels] = {0}, bnd_begin[kMaxLevels] = {0};
  int64_t n_ops = 0, n_ops_bf16 = 0;
};

struct PointSet {
  int64_t n = 0;
  int64_t *pos = nullptr;      // sorted positions (recording)
  float *interp = nullptr;     // n x Np Lagrange values (recording)
  float *w = nullptr;          // n x Np delta weights (injection)
  int *start = nullptr, *count = nullptr, *point = nullptr;  // CSR over sorted positions
  int *eflag = nullptr;        // mesh flags | 4 where points inject
};

struct Field {
  float *q = nullptr, *ring = nullptr, *tr = nullptr;
  int64_t tau = 0;
};

struct dgrtm_shot_s {
  dgrtm_mesh mesh = nullptr;
  dgrtm_shot_args args{};
  int64_t n_global = 0;
  int n_local = 1;
  int64_t C = 1, n_ckpt = 0;
  Field S, R;
  double *img = nullptr;
  float *ckpt = nullptr;
  float *seg_q = nullptr, *seg_r = nullptr;
  int64_t seg_q_off[kMaxLevels] = {0}, seg_r_off[kMaxLevels] = {0};
  PointSet src, rec;
  float *wavelet = nullptr;
  float *traces = nullptr;     // n_rec x (n_global + 1)
  double *red = nullptr;       // FP64 reduction scratch
  // boundary-trace storage (DGRTM_STORE_BOUNDARY): the record, and the states at the starts of
  // the last two global steps (index 0: global time NG - 1, index 1: NG - 2)
  bool replay = false;
  float *bnd_rec = nullptr;
  int64_t bnd_off[kMaxLevels] = {0};
  float *qsave[2] = {nullptr, nullptr};
  bool trapezoid = false;
  bool forward_done = false;
  // pipeline state, advanced one global step at a time (dgrtm_step_shots)
  int ph = DGRTM_PHASE_IDLE;
  int64_t g = 0;               // forward / recompute: next global step of the source field
  int64_t c = 0, g0 = 0, g1 = 0;  // adjoint: current segment [g0, g1)
  int64_t gr = 0, gr_end = 0;  // adjoint: next / last+1 global step of the receiver field in this segment
  bool full_rtm = false;       // run the adjoint right after the forward (serving)
  const float *data = nullptr;
  int condition = DGRTM_IMAGE_CHARACTERISTIC;
  float up[3] = {0.f, 0.f, 1.f};
  int64_t g_image_start = 0;
  // sampled HIP-event timing of the step kernel (dgrtm_profile_*)
  int prof_every = 0;
  int64_t prof_counter = 0;
  std::vector<hipEvent_t> prof_ev;
  struct ProfRec {
    int mode;
    int64_t elems;
    size_t ev;
  };
  std::vector<ProfRec> prof_rec;
  ~dgrtm_shot_s() {
    for (auto e : prof_ev) (void)hipEventDestroy(e);
  }
};

static int64_t level_end_h(const HostMesh &m, int l) { return l == 1 ? m.lev_begin[m.L] : m.lev_begin[l - 2]; }
static int64_t level_size_h(const HostMesh &m, int l) { return level_end_h(m, l) - m.lev_begin[l - 1]; }

extern "C" const char *dgrtm_last_error(void) { return g_err.c_str(); }

extern "C" dgrtm_status dgrtm_mesh_create(int N, int64_t n_vert, const double *vert_xyz, int64_t n_elem,
                                          const int64_t *elem_vert, const int8_t *face_bc, int bc_default,
                                          dgrtm_mesh *out) {
  if (!out || N < 1 || N > 6 || n_vert < 4 || n_elem < 1 || !vert_xyz || !elem_vert)
    return fail(DGRTM_ERR_ARG, "dgrtm_mesh_create: bad argument (N must be 1..6)");
  if (n_elem > (int64_t)1 << 30) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_create: too many elements");
  if (!face_bc && (bc_default < 1 || bc_default > 3)) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_create: bad bc_default");
  auto *m = new dgrtm_mesh_s();
  build_ref(N, m->ref);
  std::string err = mesh_build(m->hm, N, n_vert, vert_xyz, n_elem, elem_vert, face_bc, bc_default, m->ref);
  if (!err.empty()) {
    delete m;
    return fail(DGRTM_ERR_MESH, "dgrtm_mesh_create: " + err);
  }
  *out = m;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_set_model(dgrtm_mesh m, const double *rho, const double *c, int n_levels_max,
                                        double cfl, double *dt_local_out, int *n_levels_out) {
  if (!m || !rho || !c || !(cfl > 0)) return fail(DGRTM_ERR_ARG, "dgrtm_set_model: bad argument");
  if (m->bound) return fail(DGRTM_ERR_ARG, "dgrtm_set_model: mesh already bound");
  std::string err = mesh_set_model(m->hm, rho, c, n_levels_max, cfl);
  if (!err.empty()) return fail(DGRTM_ERR_ARG, "dgrtm_set_model: " + err);
  if (dt_local_out) *dt_local_out = m->hm.dt_local;
  if (n_levels_out) *n_levels_out = m->hm.L;
  return DGRTM_OK;
}

static size_t mesh_layout(dgrtm_mesh m, Bump &b) {
  const HostMesh &h = m->hm;
  const int64_t K = h.Ktot;
  const int64_t n_ops = op_fragment_floats(m->ref.N);
  float *geo = b.take<float>((size_t)kGeo * K);
  int *nbr = b.take<int>((size_t)4 * K);
  int *ncode = b.take<int>((size_t)4 * K);
  int *eflag = b.take<int>((size_t)K);
  float *ops = b.take<float>((size_t)n_ops);
  const int64_t n_ops_bf16 = op_fragment_bf16_words(m->ref.N);
  uint32_t *ops_bf16 = b.take<uint32_t>((size_t)n_ops_bf16);
  int8_t *nidx = b.take<int8_t>((size_t)4 * 4 * 6 * m->ref.Nfp);
  int64_t *s2u = b.take<int64_t>((size_t)K);
  uint32_t *tctr = b.take<uint32_t>((size_t)2 * kMaxSlots);
  int64_t nbf = 0;
  for (int64_t i = 0; i < 4 * h.K; ++i) nbf += h.bc[i] != 0;
  int *bface = b.take<int>((size_t)std::max<int64_t>(nbf, 1));
  if (b.base) {  // a sizing pass (no base) leaves the handle untouched
    m->bface = bface;
    m->n_bfaces = nbf;
    m->geo = geo;
    m->nbr = nbr;
    m->ncode = ncode;
    m->eflag = eflag;
    m->n_ops = n_ops;
    m->ops = ops;
    m->n_ops_bf16 = n_ops_bf16;
    m->ops_bf16 = ops_bf16;
    m->nbr_index = nidx;
    m->s2u = s2u;
    m->tile_ctr = tctr;
  }
  return b.used;
}

extern "C" dgrtm_status dgrtm_mesh_bytes(dgrtm_mesh m, size_t *bytes) {
  if (!m || !bytes) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_bytes: bad argument");
  if (!m->hm.has_model) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_bytes: call dgrtm_set_model first");
  Bump b;
  *bytes = mesh_layout(m, b) + 256;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_mesh_bind(dgrtm_mesh m, void *dev_ws, size_t ws_bytes, void *hip_stream) {
  if (!m || !dev_ws) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_bind: bad argument");
  if (!m->hm.has_model) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_bind: call dgrtm_set_model first");
  if (((uintptr_t)dev_ws) % 256) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_bind: workspace must be 256-byte aligned");
  Bump probe;
  size_t need = mesh_layout(m, probe);
  if (ws_bytes < need) return fail(DGRTM_ERR_WORKSPACE, "dgrtm_mesh_bind: workspace too small");
  Bump b;
  b.base = (char *)dev_ws;
  mesh_layout(m, b);
  m->stream = (hipStream_t)hip_stream;
  const HostMesh &h = m->hm;
  const RefOps &R = m->ref;
  const int64_t K = h.Ktot;
  // geometry and material in device order; padding slots get an identity metric and unit material
  std::vector<float> geo((size_t)kGeo * K, 0.0f);
  std::vector<int> nbr((size_t)4 * K, -2), ncode((size_t)4 * K, 0);
  m->h_eflag.assign(K, 0);
  // boundary faces in sorted order (finest level first); a boundary face's code is its index among
  // its level's boundary faces, a padding element's codes are -1
  std::vector<int> bface;
  for (int l = 0; l < kMaxLevels; ++l) m->bnd_cnt[l] = m->bnd_begin[l] = 0;
  int cur_level = -1;
  for (int64_t s = 0; s < K; ++s) {
    int64_t u = h.sorted_to_user[s];
    if (u < 0) {
      for (int f = 0; f < 4; ++f) ncode[tix(4, f, s)] = -1;
      geo[tix(kGeo, 0, s)] = geo[tix(kGeo, 4, s)] = geo[tix(kGeo, 8, s)] = 1.0f;
      geo[tix(kGeo, 9, s)] = geo[tix(kGeo, 10, s)] = geo[tix(kGeo, 11, s)] = 1.0f;
      continue;
    }
    for (int i = 0; i < 9; ++i) geo[tix(kGeo, i, s)] = (float)h.geo[9 * u + i];
    const double Zm = h.rho[u] * h.c[u];
    geo[tix(kGeo, 9, s)] = (float)(h.rho[u] * h.c[u] * h.c[u]);
    geo[tix(kGeo, 10, s)] = (float)(1.0 / h.rho[u]);
    geo[tix(kGeo, 11, s)] = (float)Zm;
    int flag = 1;
    for (int f = 0; f < 4; ++f) {
      const int64_t u2 = h.EToE[4 * u + f];
      const int b_ = h.bc[4 * u + f];
      double taup, tauv;
      if (b_ != 0) {
        taup = 1.0 / Zm;
        tauv = Zm;
        nbr[tix(4, f, s)] = -b_;
        const int lv = h.level[u];
        if (lv != cur_level) {
          cur_level = lv;
          m->bnd_begin[lv - 1] = (int64_t)bface.size();
        }
        ncode[tix(4, f, s)] = (int)m->bnd_cnt[lv - 1]++;
        bface.push_back((int)(s * 4 + f));
      } else {
        const double Zp = h.rho[u2] * h.c[u2];
        taup = 2.0 / (Zm + Zp);
        tauv = 0.5 * (Zm + Zp);
        nbr[tix(4, f, s)] = (int)h.user_to_sorted[u2];
        ncode[tix(4, f, s)] = h.EToF[4 * u + f] | (h.face_perm[4 * u + f] << 2) | (h.level[u2] << 5);
        if (h.level[u2] > h.level[u]) flag |= 2;
      }
      geo[tix(kGeo, 12 + f, s)] = (float)taup;
      geo[tix(kGeo, 16 + f, s)] = (float)tauv;
    }
    m->h_eflag[s] = flag;
  }
  const int Np = R.Np, F = 4 * R.Nfp;
  std::vector<float> Dr(Np * Np), Ds(Np * Np), Dt(Np * Np), L(Np * F);
  for (int i = 0; i < Np * Np; ++i) {
    Dr[i] = (float)R.Dr[i];
    Ds[i] = (float)R.Ds[i];
    Dt[i] = (float)R.Dt[i];
  }
  for (int i = 0; i < Np * F; ++i) L[i] = (float)R.LIFT[i];
  std::vector<float> frag(m->n_ops);
  build_op_fragments(R.N, Dr.data(), Ds.data(), Dt.data(), L.data(), frag.data());
  std::vector<uint32_t> fragb(m->n_ops_bf16);
  build_op_fragments_bf16(R.N, R.Dr.data(), R.Ds.data(), R.Dt.data(), R.LIFT.data(), fragb.data());
  std::vector<int8_t> nidx(R.nbr_index.size());
  for (size_t i = 0; i < nidx.size(); ++i) nidx[i] = (int8_t)R.nbr_index[i];
  hipStream_t st = m->stream;
  HIPCHK(hipMemcpyAsync(m->geo, geo.data(), geo.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->ncode, ncode.data(), ncode.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->eflag, m->h_eflag.data(), K * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->ops, frag.data(), frag.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->ops_bf16, fragb.data(), fragb.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->nbr_index, nidx.data(), nidx.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(m->s2u, h.sorted_to_user.data(), K * 8, hipMemcpyHostToDevice, st));
  if ((int64_t)bface.size() != m->n_bfaces) return fail(DGRTM_ERR_MESH, "dgrtm_mesh_bind: boundary face count");
  if (!bface.empty())
    HIPCHK(hipMemcpyAsync(m->bface, bface.data(), bface.size() * 4, hipMemcpyHostToDevice, st));
  // the step kernel leaves its counters at zero when it ends; they start at zero here
  const std::vector<uint32_t> zero(2 * kMaxSlots, 0u);
  HIPCHK(hipMemcpyAsync(m->tile_ctr, zero.data(), zero.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  m->bound = true;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_mesh_set_launch_cap(dgrtm_mesh m, int64_t max_groups) {
  if (!m || max_groups < 0) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_set_launch_cap: bad argument");
  m->max_groups = max_groups;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_export_setup(dgrtm_mesh m, int32_t *EToE, int8_t *EToF, int32_t *vmapP, int8_t *level,
                                           int64_t *sorted_pos) {
  if (!m) return fail(DGRTM_ERR_ARG, "dgrtm_export_setup: bad argument");
  const HostMesh &h = m->hm;
  if (EToE) std::copy(h.EToE.begin(), h.EToE.end(), EToE);
  if (EToF) std::copy(h.EToF.begin(), h.EToF.end(), EToF);
  if (vmapP) mesh_vmapP(h, m->ref, vmapP);
  if (level || sorted_pos) {
    if (!h.has_model) return fail(DGRTM_ERR_ARG, "dgrtm_export_setup: levels need dgrtm_set_model");
    if (level) std::copy(h.level.begin(), h.level.end(), level);
    if (sorted_pos) std::copy(h.user_to_sorted.begin(), h.user_to_sorted.end(), sorted_pos);
  }
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_locate(dgrtm_mesh m, int64_t n, const double *xyz, int64_t *elem) {
  if (!m || n < 0 || (n > 0 && (!xyz || !elem))) return fail(DGRTM_ERR_ARG, "dgrtm_locate: bad argument");
  std::vector<double> rst(3 * (size_t)std::max<int64_t>(n, 1));
  if (n) locate_points(m->hm, n, xyz, elem, rst.data());
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_export_operators(dgrtm_mesh m, double *Dr, double *Ds, double *Dt, double *LIFT,
                                               double *rst) {
  if (!m) return fail(DGRTM_ERR_ARG, "dgrtm_export_operators: bad argument");
  const RefOps &R = m->ref;
  if (Dr) std::copy(R.Dr.begin(), R.Dr.end(), Dr);
  if (Ds) std::copy(R.Ds.begin(), R.Ds.end(), Ds);
  if (Dt) std::copy(R.Dt.begin(), R.Dt.end(), Dt);
  if (LIFT) std::copy(R.LIFT.begin(), R.LIFT.end(), LIFT);
  if (rst)
    for (int n = 0; n < R.Np; ++n) {
      rst[3 * n] = R.r[n];
      rst[3 * n + 1] = R.s[n];
      rst[3 * n + 2] = R.t[n];
    }
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_mesh_info(dgrtm_mesh m, int *N, int *Np, int *Nfp, int64_t *n_elem, int *n_levels,
                                        double *dt_local) {
  if (!m) return fail(DGRTM_ERR_ARG, "dgrtm_mesh_info: bad argument");
  if (N) *N = m->ref.N;
  if (Np) *Np = m->ref.Np;
  if (Nfp) *Nfp = m->ref.Nfp;
  if (n_elem) *n_elem = m->hm.K;
  if (n_levels) *n_levels = m->hm.L;
  if (dt_local) *dt_local = m->hm.dt_local;
  return DGRTM_OK;
}

extern "C" void dgrtm_mesh_destroy(dgrtm_mesh m) { delete m; }

// ------------------------------------------------------------------------------------------------
// shots
// ------------------------------------------------------------------------------------------------
static dgrtm_status check_args(dgrtm_mesh m, const dgrtm_shot_args *a) {
  if (!m || !a) return fail(DGRTM_ERR_ARG, "bad argument");
  if (a->struct_size != (int32_t)sizeof(dgrtm_shot_args)) return fail(DGRTM_ERR_ARG, "dgrtm_shot_args: struct_size mismatch");
  if (!m->hm.has_model) return fail(DGRTM_ERR_ARG, "call dgrtm_set_model first");
  if (!(a->t_final > 0)) return fail(DGRTM_ERR_ARG, "t_final must be positive");
  if (a->n_rec < 0 || (a->n_rec > 0 && !a->rec_xyz)) return fail(DGRTM_ERR_ARG, "bad receivers");
  if (a->ckpt_interval < 0) return fail(DGRTM_ERR_ARG, "bad ckpt_interval");
  if (a->precision != DGRTM_FP32 && a->precision != DGRTM_SPLIT_BF16) return fail(DGRTM_ERR_ARG, "bad precision");
  if (a->storage != DGRTM_STORE_CHECKPOINTS && a->storage != DGRTM_STORE_BOUNDARY)
    return fail(DGRTM_ERR_ARG, "bad storage");
  return DGRTM_OK;
}

static void shot_steps(dgrtm_mesh m, const dgrtm_shot_args *a, int64_t &ng, int &nl) {
  nl = 1 << (m->hm.L - 1);
  const double dtg = m->hm.dt_local * nl;
  ng = std::max<int64_t>(1, (int64_t)std::ceil(a->t_final / dtg - 1e-9));
}

extern "C" dgrtm_status dgrtm_shot_steps(dgrtm_mesh m, const dgrtm_shot_args *a, int64_t *n_global, int32_t *n_local) {
  dgrtm_status s = check_args(m, a);
  if (s) return s;
  int64_t ng;
  int nl;
  shot_steps(m, a, ng, nl);
  if (n_global) *n_global = ng;
  if (n_local) *n_local = nl;
  return DGRTM_OK;
}

static int64_t choose_interval(dgrtm_mesh m, const dgrtm_shot_args *a, int64_t ng) {
  if (a->storage == DGRTM_STORE_BOUNDARY) return 1;   // segment records of one global step at a time
  if (a->ckpt_interval > 0) return std::min(a->ckpt_interval, ng);
  const HostMesh &h = m->hm;
  const int Np = m->ref.Np;
  double ck = 3.0 * state_row(Np) * h.Ktot;
  double seg = 0;
  for (int l = 1; l <= h.L; ++l) seg += 2.0 * Np * (double)level_size_h(h, l) * (1 << (l - 1));
  int64_t C = (int64_t)std::llround(std::sqrt((double)ng * ck / std::max(seg, 1.0)));
  return std::min<int64_t>(std::max<int64_t>(C, 1), ng);
}

// boundary faces per level (index l - 1)
static void boundary_counts(const HostMesh &h, int64_t *cnt) {
  for (int l = 0; l < kMaxLevels; ++l) cnt[l] = 0;
  for (int64_t u = 0; u < h.K; ++u)
    for (int f = 0; f < 4; ++f)
      if (h.bc[4 * u + f] != 0) ++cnt[h.level[u] - 1];
}

static size_t shot_layout(dgrtm_shot sh, Bump &b) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  const int Np = m->ref.Np, F = 4 * m->ref.Nfp;
  const int64_t K = h.Ktot;
  for (Field *f : {&sh->S, &sh->R}) {
    f->q = b.take<float>((size_t)state_row(Np) * K);
    f->ring = b.take<float>((size_t)3 * state_row(Np) * K);
    f->tr = b.take<float>((size_t)3 * trace_row(m->ref.Nfp) * K);
  }
  sh->img = b.take<double>((size_t)Np * K);
  sh->ckpt = b.take<float>((size_t)sh->n_ckpt * 3 * state_row(Np) * K);
  if (sh->replay) {
    // level l: rows j = 0 .. NG 2^(l-1) of its boundary faces, 2 FS floats each
    const int64_t row = 2 * trace_face_stride(m->ref.Nfp);
    int64_t cnt[kMaxLevels], off = 0;
    boundary_counts(h, cnt);
    for (int l = 1; l <= h.L; ++l) {
      sh->bnd_off[l - 1] = off;
      off += ((sh->n_global << (l - 1)) + 1) * cnt[l - 1] * row;
    }
    sh->bnd_rec = b.take<float>((size_t)std::max<int64_t>(off, 4));
    for (int i = 0; i < 2; ++i) sh->qsave[i] = b.take<float>((size_t)state_row(Np) * K);
  }
  int64_t oq = 0, orr = 0;
  for (int l = 1; l <= h.L; ++l) {
    const int64_t P = level_size_h(h, l), nst = sh->C * ((int64_t)1 << (l - 1));
    sh->seg_q_off[l - 1] = oq;
    sh->seg_r_off[l - 1] = orr;
    oq += nst * Np * P;
    orr += (nst + 2) * Np * P;
  }
  sh->seg_q = b.take<float>((size_t)oq);
  sh->seg_r = b.take<float>((size_t)orr);
  for (PointSet *p : {&sh->src, &sh->rec}) {
    p->pos = b.take<int64_t>((size_t)std::max<int64_t>(p->n, 1));
    p->interp = b.take<float>((size_t)std::max<int64_t>(p->n, 1) * Np);
    p->w = b.take<float>((size_t)std::max<int64_t>(p->n, 1) * Np);
    p->start = b.take<int>((size_t)K);
    p->count = b.take<int>((size_t)K);
    p->point = b.take<int>((size_t)std::max<int64_t>(p->n, 1));
    p->eflag = b.take<int>((size_t)K);
  }
  sh->wavelet = b.take<float>((size_t)sh->n_global * sh->n_local + 1);
  sh->traces = b.take<float>((size_t)std::max<int64_t>(sh->rec.n, 1) * (sh->n_global + 1));
  sh->red = b.take<double>(8);
  return b.used;
}

static dgrtm_shot new_shot(dgrtm_mesh m, const dgrtm_shot_args *a) {
  auto *sh = new dgrtm_shot_s();
  sh->mesh = m;
  sh->args = *a;
  shot_steps(m, a, sh->n_global, sh->n_local);
  sh->replay = a->storage == DGRTM_STORE_BOUNDARY;
  sh->C = choose_interval(m, a, sh->n_global);
  sh->n_ckpt = sh->replay ? 0 : (sh->n_global + sh->C - 1) / sh->C;
  sh->src.n = a->has_source ? 1 : 0;
  sh->rec.n = a->n_rec;
  return sh;
}

extern "C" dgrtm_status dgrtm_shot_bytes(dgrtm_mesh m, const dgrtm_shot_args *a, size_t *bytes) {
  dgrtm_status s = check_args(m, a);
  if (s) return s;
  if (!bytes) return fail(DGRTM_ERR_ARG, "dgrtm_shot_bytes: bad argument");
  dgrtm_shot sh = new_shot(m, a);
  Bump b;
  *bytes = shot_layout(sh, b) + 256;
  delete sh;
  return DGRTM_OK;
}

// locate points, build per-point interpolation rows / delta weights and the CSR lists
static dgrtm_status upload_points(dgrtm_shot sh, PointSet &p, const double *xyz) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  const RefOps &R = m->ref;
  const int Np = R.Np;
  const int64_t K = h.Ktot;
  std::vector<int64_t> elem(p.n);
  std::vector<double> rst(3 * p.n);
  if (p.n) locate_points(h, p.n, xyz, elem.data(), rst.data());
  std::vector<double> Vt(Np * Np);  // V^T for solving l = V^{-T} psi
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) Vt[i * Np + j] = R.V[j * Np + i];
  std::vector<double> Vti = Vt;
  invert(Np, Vti);
  std::vector<float> interp(std::max<int64_t>(p.n, 1) * Np), w(std::max<int64_t>(p.n, 1) * Np);
  std::vector<int64_t> pos(std::max<int64_t>(p.n, 1), 0);
  std::vector<double> psi(Np);
  for (int64_t i = 0; i < p.n; ++i) {
    if (elem[i] < 0) return fail(DGRTM_ERR_OUTSIDE, "point " + std::to_string(i) + " lies outside the mesh");
    basis_at(R, rst[3 * i], rst[3 * i + 1], rst[3 * i + 2], psi.data());
    pos[i] = h.user_to_sorted[elem[i]];
    const double J = h.J[elem[i]];
    for (int n = 0; n < Np; ++n) {
      double l = 0.0, wv = 0.0;
      for (int j = 0; j < Np; ++j) {
        l += Vti[n * Np + j] * psi[j];
        wv += R.V[n * Np + j] * psi[j];
      }
      interp[i * Np + n] = (float)l;
      w[i * Np + n] = (float)(wv / J);  // M_k^{-1} l(x0) = (1/J) V psi(r0)
    }
  }
  // CSR: points grouped by sorted position
  std::vector<int> start(K, 0), count(K, 0), point(std::max<int64_t>(p.n, 1), 0);
  for (int64_t i = 0; i < p.n; ++i) count[pos[i]]++;
  int acc = 0;
  for (int64_t s = 0; s < K; ++s) {
    start[s] = acc;
    acc += count[s];
  }
  std::vector<int> fill(start);
  for (int64_t i = 0; i < p.n; ++i) point[fill[pos[i]]++] = (int)i;
  std::vector<int> ef(m->h_eflag);
  for (int64_t s = 0; s < K; ++s)
    if (count[s]) ef[s] |= 4;
  hipStream_t st = m->stream;
  HIPCHK(hipMemcpyAsync(p.pos, pos.data(), pos.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.interp, interp.data(), interp.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.w, w.data(), w.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.start, start.data(), K * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.count, count.data(), K * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.point, point.data(), point.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.eflag, ef.data(), K * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_shot_create(dgrtm_mesh m, const dgrtm_shot_args *a, void *dev_ws, size_t ws_bytes,
                                          dgrtm_shot *out) {
  dgrtm_status s = check_args(m, a);
  if (s) return s;
  if (!out || !dev_ws) return fail(DGRTM_ERR_ARG, "dgrtm_shot_create: bad argument");
  if (!m->bound) return fail(DGRTM_ERR_ARG, "dgrtm_shot_create: mesh not bound");
  if (((uintptr_t)dev_ws) % 256) return fail(DGRTM_ERR_ARG, "dgrtm_shot_create: workspace must be 256-byte aligned");
  dgrtm_shot sh = new_shot(m, a);
  Bump probe;
  if (ws_bytes < shot_layout(sh, probe)) {
    delete sh;
    return fail(DGRTM_ERR_WORKSPACE, "dgrtm_shot_create: workspace too small");
  }
  Bump b;
  b.base = (char *)dev_ws;
  shot_layout(sh, b);
  if ((s = upload_points(sh, sh->src, a->src_xyz)) || (s = upload_points(sh, sh->rec, a->rec_xyz))) {
    delete sh;
    return s;
  }
  // source signal at every local step (FP64 on the host, stored FP32)
  const int64_t nst = sh->n_global * sh->n_local + 1;
  std::vector<float> wav(nst, 0.0f);
  for (int64_t j = 0; j < nst; ++j) {
    if (a->wavelet) wav[j] = a->wavelet[j];
    else {
      const double t = j * m->hm.dt_local;
      const double x = M_PI * a->f_peak * (t - a->t_peak);
      wav[j] = (float)(a->amp * (1.0 - 2.0 * x * x) * std::exp(-x * x));
    }
  }
  hipStream_t st = m->stream;
  hipError_t e = hipMemcpyAsync(sh->wavelet, wav.data(), nst * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete sh;
    return fail(DGRTM_ERR_HIP, std::string("dgrtm_shot_create: ") + hipGetErrorString(e));
  }
  *out = sh;
  return DGRTM_OK;
}

extern "C" void dgrtm_shot_destroy(dgrtm_shot sh) { delete sh; }

// ------------------------------------------------------------------------------------------------
// time stepping
// ------------------------------------------------------------------------------------------------
static void fill_level_begin(const HostMesh &h, int64_t *lb) {
  for (int i = 0; i <= kMaxLevels; ++i) lb[i] = 0;
  for (int l = 0; l <= h.L; ++l) lb[l] = h.lev_begin[l];
}

static StepArgs mesh_args(dgrtm_mesh m, int precision, int mode, bool reversed, int n_local) {
  const HostMesh &h = m->hm;
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.geo = m->geo;
  a.nbr = m->nbr;
  a.ncode = m->ncode;
  a.ops = m->ops;
  a.ops_bf16 = m->ops_bf16;
  a.nbr_index = m->nbr_index;
  a.tile_ctr = m->tile_ctr;
  a.max_groups = m->max_groups;
  a.Ktot = h.Ktot;
  a.L = h.L;
  fill_level_begin(h, a.lev_begin);
  for (int l = 0; l < kMaxLevels; ++l) a.bnd_cnt[l] = m->bnd_cnt[l];
  a.dt_local = h.dt_local;
  a.tau_sign = reversed ? -1.0f : 1.0f;
  a.out_sign = reversed ? -1.0f : 1.0f;
  a.n_local = n_local;
  a.precision = precision;
  a.mode = mode;
  return a;
}

// end of the active prefix at local step tau: levels whose step starts at tau
static int64_t active_end(const HostMesh &h, int64_t tau) {
  for (int l = 1; l <= h.L; ++l)
    if ((tau & (((int64_t)1 << (h.L - l)) - 1)) == 0) return level_end_h(h, l);
  return level_end_h(h, h.L);
}

// real elements in the active prefix [0, k_end)
static int64_t active_elements(const HostMesh &h, int64_t k_end) {
  int64_t n = 0;
  for (int l = 1; l <= h.L; ++l)
    if (h.lev_begin[l - 1] < k_end) n += h.lev_count[l - 1];
  return n;
}

static dgrtm_status trace_init(dgrtm_shot sh, Field &f) {
  dgrtm_mesh m = sh->mesh;
  TraceInitArgs t;
  std::memset(&t, 0, sizeof(t));
  t.q = f.q;
  t.tr = f.tr;
  t.geo = m->geo;
  t.eflag = m->eflag;
  t.Ktot = m->hm.Ktot;
  t.L = m->hm.L;
  fill_level_begin(m->hm, t.lev_begin);
  t.tau = f.tau;
  HIPCHK(launch_trace_init(m->ref.N, t, m->stream));
  return DGRTM_OK;
}

static dgrtm_status zero_field(dgrtm_shot sh, Field &f) {
  dgrtm_mesh m = sh->mesh;
  const int Np = m->ref.Np, F = 4 * m->ref.Nfp;
  const int64_t K = m->hm.Ktot;
  HIPCHK(launch_fill_f32(f.q, (int64_t)state_row(Np) * K, 0.0f, m->stream));
  HIPCHK(launch_fill_f32(f.ring, 3LL * state_row(Np) * K, 0.0f, m->stream));
  HIPCHK(launch_fill_f32(f.tr, 3LL * trace_row(m->ref.Nfp) * K, 0.0f, m->stream));
  f.tau = 0;
  return DGRTM_OK;
}

// Launch one local step for `n` slots (same mesh, mode and local phase), timing it if sampled.
static dgrtm_status launch_slots(dgrtm_shot prof_owner, StepArgs &a, int64_t tau) {
  dgrtm_mesh m = prof_owner->mesh;
  a.k_end = active_end(m->hm, tau);
  dgrtm_shot sh = prof_owner;
  const bool prof = sh->prof_every > 0 && (sh->prof_counter++ % sh->prof_every) == 0;
  size_t ev = 0;
  if (prof) {
    ev = sh->prof_rec.size() * 2;
    while (sh->prof_ev.size() < ev + 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      sh->prof_ev.push_back(e);
    }
    HIPCHK(hipEventRecord(sh->prof_ev[ev], m->stream));
  }
  HIPCHK(launch_step(m->ref.N, a, m->stream));
  if (prof) {
    HIPCHK(hipEventRecord(sh->prof_ev[ev + 1], m->stream));
    sh->prof_rec.push_back({a.mode, active_elements(m->hm, a.k_end) * a.nslots, ev});
  }
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_profile_start(dgrtm_shot sh, int sample_every) {
  if (!sh || sample_every < 0) return fail(DGRTM_ERR_ARG, "dgrtm_profile_start: bad argument");
  sh->prof_every = sample_every;
  sh->prof_counter = 0;
  sh->prof_rec.clear();
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_profile_read(dgrtm_shot sh, int mode, double *kernel_ms, int64_t *launches,
                                           int64_t *element_steps) {
  if (!sh || mode < 0 || mode > 4) return fail(DGRTM_ERR_ARG, "dgrtm_profile_read: bad argument");
  HIPCHK(hipStreamSynchronize(sh->mesh->stream));
  double ms = 0.0;
  int64_t n = 0, es = 0;
  for (const auto &r : sh->prof_rec) {
    if (r.mode != mode) continue;
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, sh->prof_ev[r.ev], sh->prof_ev[r.ev + 1]));
    ms += t;
    ++n;
    es += r.elems;
  }
  if (kernel_ms) *kernel_ms = ms;
  if (launches) *launches = n;
  if (element_steps) *element_steps = es;
  return DGRTM_OK;
}

static SlotArgs field_slot(dgrtm_shot sh, Field &f) {
  SlotArgs s;
  std::memset(&s, 0, sizeof(s));
  s.q = f.q;
  s.ring = f.ring;
  s.tr = f.tr;
  s.eflag = sh->mesh->eflag;
  s.tau = f.tau;
  s.up[2] = 1.0f;
  s.src_scale = 1.0f;
  s.C = sh->C;
  s.NG = sh->n_global;
  return s;
}

static void with_points(SlotArgs &s, const PointSet &p, int amp_mode) {
  if (p.n == 0) return;
  s.eflag = p.eflag;
  s.src_start = p.start;
  s.src_count = p.count;
  s.src_point = p.point;
  s.src_w = p.w;
  s.amp_mode = amp_mode;
}

// the slot of a shot for its next global step, and the step mode
static SlotArgs phase_slot(dgrtm_shot sh, int &mode, bool &reversed, Field *&field) {
  SlotArgs s;
  if (sh->ph == DGRTM_PHASE_BACKWARD) {
    field = &sh->R;
    s = field_slot(sh, sh->R);
    with_points(s, sh->rec, 1);
    s.data = sh->data ? sh->data : sh->traces;
    s.n_t = sh->n_global + 1;
    s.src_scale = -1.0f;
    s.seg_q = sh->seg_q;
    s.seg_r = sh->seg_r;
    s.img = sh->img;
    s.g0 = sh->g0;
    s.g1 = sh->g1;
    s.image_from = sh->g_image_start * sh->n_local;
    s.img_rule = sh->trapezoid ? IMG_TRAPEZOID : 0;
    if (sh->replay) {   // both fields run backward: the source record is at the same own step
      s.img_rule |= IMG_SAME_DIR;
      s.image_from = 0;
    }
    mode = MODE_IMAGE;
    reversed = true;
  } else if (sh->ph == DGRTM_PHASE_RECOMPUTE && sh->replay) {
    // the source field re-simulated backward in time with the recorded boundary traces
    field = &sh->S;
    s = field_slot(sh, sh->S);
    if (sh->args.has_source) with_points(s, sh->src, 2);
    s.wavelet = sh->wavelet;
    s.n_t = sh->n_global * sh->n_local + 1;
    s.src_scale = -1.0f;
    s.bnd_rec = sh->bnd_rec;
    std::memcpy(s.bnd_off, sh->bnd_off, sizeof(s.bnd_off));
    s.seg_q = sh->seg_q;
    s.seg_r = sh->seg_r;
    s.g0 = sh->g0;
    s.g1 = sh->g1;
    mode = MODE_REPLAY_SEG;
    reversed = true;
  } else {
    field = &sh->S;
    s = field_slot(sh, sh->S);
    if (sh->args.has_source) with_points(s, sh->src, 0);
    s.wavelet = sh->wavelet;
    mode = MODE_PLAIN;
    reversed = false;
    if (sh->ph == DGRTM_PHASE_RECOMPUTE) {
      s.seg_q = sh->seg_q;
      s.seg_r = sh->seg_r;
      s.g0 = sh->g0;
      s.g1 = sh->g1;
      mode = MODE_RECORD_SEG;
    }
  }
  std::memcpy(s.up, sh->up, sizeof(s.up));
  s.condition = sh->condition;
  return s;
}

static dgrtm_status record(dgrtm_shot sh, Field &f, int64_t g) {
  dgrtm_mesh m = sh->mesh;
  HIPCHK(launch_record(m->ref.N, f.q, m->hm.Ktot, sh->rec.pos, sh->rec.interp, sh->rec.n, sh->traces + g,
                       sh->n_global + 1, m->stream));
  return DGRTM_OK;
}

// checkpoint c = state at the start of global step c*C: q and the two newest rhs of every level
static dgrtm_status ckpt_copy(dgrtm_shot sh, Field &f, int64_t c, bool save) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  const int Np = m->ref.Np;
  const int64_t K = h.Ktot, slab = (int64_t)state_row(Np) * K;
  float *ck = sh->ckpt + c * 3 * slab;
  const int64_t g = c * sh->C;
  hipStream_t st = m->stream;
  if (save) HIPCHK(hipMemcpyAsync(ck, f.q, slab * 4, hipMemcpyDeviceToDevice, st));
  else HIPCHK(hipMemcpyAsync(f.q, ck, slab * 4, hipMemcpyDeviceToDevice, st));
  for (int l = 1; l <= h.L; ++l) {
    const int64_t mstep = g << (l - 1);
    const int64_t b0 = h.lev_begin[l - 1], P = level_size_h(h, l);
    if (P == 0) continue;
    for (int s = 1; s <= 2; ++s) {
      // a level is a whole number of tiles, hence one contiguous block of the tiled layout
      const int64_t slot = ((mstep - s) % 3 + 3) % 3;
      float *ring = f.ring + slot * slab + b0 * state_row(Np);
      float *cks = ck + s * slab + b0 * state_row(Np);
      const size_t bytes = (size_t)P * state_row(Np) * sizeof(float);
      if (save) HIPCHK(hipMemcpyAsync(cks, ring, bytes, hipMemcpyDeviceToDevice, st));
      else HIPCHK(hipMemcpyAsync(ring, cks, bytes, hipMemcpyDeviceToDevice, st));
    }
  }
  return DGRTM_OK;
}

// start segment c of the adjoint: restore S at g0 and prepare its segment buffer history
static dgrtm_status begin_segment(dgrtm_shot sh, int64_t c) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  dgrtm_status s;
  sh->c = c;
  sh->g0 = c * sh->C;
  sh->g1 = std::min(sh->n_global, sh->g0 + sh->C);
  sh->g = sh->g0;
  if ((s = ckpt_copy(sh, sh->S, c, false))) return s;
  sh->S.tau = sh->g0 * sh->n_local;
  if ((s = trace_init(sh, sh->S))) return s;
  SegInitArgs si;
  std::memset(&si, 0, sizeof(si));
  si.ring = sh->S.ring;
  si.geo = m->geo;
  si.eflag = m->eflag;
  si.seg_r = sh->seg_r;
  si.Ktot = h.Ktot;
  si.L = h.L;
  fill_level_begin(h, si.lev_begin);
  std::memcpy(si.up, sh->up, sizeof(si.up));
  si.condition = sh->condition;
  for (int l = 1; l <= h.L; ++l) {
    si.seg_r_off[l - 1] = sh->seg_r_off[l - 1];
    si.seg_m0[l - 1] = sh->g0 << (l - 1);
  }
  HIPCHK(launch_seg_init(m->ref.N, si, m->stream));
  sh->gr = sh->n_global - sh->g1;
  sh->gr_end = sh->n_global - std::max(sh->g0, sh->g_image_start);
  sh->ph = DGRTM_PHASE_RECOMPUTE;
  return DGRTM_OK;
}

static dgrtm_status begin_forward(dgrtm_shot sh) {
  dgrtm_status s;
  if ((s = zero_field(sh, sh->S))) return s;
  if (sh->replay) {   // row 0 of the boundary record: the traces of the state at rest
    dgrtm_mesh m = sh->mesh;
    const int64_t row = 2 * trace_face_stride(m->ref.Nfp);
    for (int l = 1; l <= m->hm.L; ++l)
      HIPCHK(launch_fill_f32(sh->bnd_rec + sh->bnd_off[l - 1], m->bnd_cnt[l - 1] * row, 0.0f, m->stream));
  }
  if ((s = record(sh, sh->S, 0))) return s;
  sh->g = 0;
  sh->forward_done = false;
  sh->ph = DGRTM_PHASE_FORWARD;
  return DGRTM_OK;
}

// segment gb of a replay adjoint: backward global step gb of the source field, recorded for the
// receiver field's image step of the same global step
static dgrtm_status begin_replay_segment(dgrtm_shot sh, int64_t gb) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  sh->c = gb;
  sh->g0 = gb;
  sh->g1 = gb + 1;
  sh->g = gb;
  if (gb > 0) {
    // The segment's two history rows per level are the r-_S rows of its first own step's two
    // predecessors, which the previous segment (the previous global step) recorded as its last
    // two rows: level l's rows 2^(l-1) and 2^(l-1) + 1 move to rows 0 and 1, one after the other
    // (at l = 1 the second source row is the first destination row's successor).
    const int Np = m->ref.Np;
    for (int l = 1; l <= h.L; ++l) {
      const int64_t P = level_size_h(h, l);
      if (P == 0) continue;
      const int64_t row = (int64_t)Np * P, n = (int64_t)1 << (l - 1);
      float *base = sh->seg_r + sh->seg_r_off[l - 1];
      for (int i = 0; i < 2; ++i)
        HIPCHK(hipMemcpyAsync(base + i * row, base + (n + i) * row, (size_t)row * sizeof(float),
                              hipMemcpyDeviceToDevice, m->stream));
    }
    sh->ph = DGRTM_PHASE_RECOMPUTE;
    return DGRTM_OK;
  }
  SegInitArgs si;
  std::memset(&si, 0, sizeof(si));
  si.ring = sh->S.ring;
  si.geo = m->geo;
  si.eflag = m->eflag;
  si.seg_r = sh->seg_r;
  si.Ktot = h.Ktot;
  si.L = h.L;
  fill_level_begin(h, si.lev_begin);
  std::memcpy(si.up, sh->up, sizeof(si.up));
  si.condition = sh->condition;
  si.history_before_start = 1;   // the extrapolated history of own steps -1 and -2
  for (int l = 1; l <= h.L; ++l) {
    si.seg_r_off[l - 1] = sh->seg_r_off[l - 1];
    si.seg_m0[l - 1] = gb << (l - 1);
  }
  HIPCHK(launch_seg_init(m->ref.N, si, m->stream));
  sh->ph = DGRTM_PHASE_RECOMPUTE;
  return DGRTM_OK;
}

// Start of a replay adjoint: the backward source run's AB3 history at t_final, extrapolated from
// its reversed-time rhs at the global times NG, NG - 1 and NG - 2 (the receiver field's buffers
// serve as scratch: state, traces, and one rhs per time in its ring), then the source field at
// its final state with own-step traces, the receiver field at rest.
static dgrtm_status begin_replay_adjoint(dgrtm_shot sh) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  const int Np = m->ref.Np;
  const int64_t K = h.Ktot, slab = (int64_t)state_row(Np) * K;
  const int nl = sh->n_local;
  dgrtm_status s;
  Field &R = sh->R;
  for (int i = 0; i < 3; ++i) {
    const int64_t G = sh->n_global - i;
    if (G < 0) {   // before t = 0 the source field is at rest and the source silent
      HIPCHK(launch_fill_f32(R.ring + i * slab, slab, 0.0f, m->stream));
      continue;
    }
    const float *q = i == 0 ? sh->S.q : sh->qsave[i - 1];
    HIPCHK(hipMemcpyAsync(R.q, q, slab * 4, hipMemcpyDeviceToDevice, m->stream));
    R.tau = i * nl;   // the backward run's local step at global time G
    if ((s = trace_init(sh, R))) return s;
    StepArgs a = mesh_args(m, sh->args.precision, MODE_RHS_REPLAY, true, nl);
    a.nslots = 1;
    a.slot[0] = field_slot(sh, R);
    if (sh->args.has_source) with_points(a.slot[0], sh->src, 2);
    a.slot[0].wavelet = sh->wavelet;
    a.slot[0].n_t = sh->n_global * nl + 1;
    a.slot[0].data_j = G * nl;
    a.slot[0].src_scale = -1.0f;
    a.slot[0].bnd_rec = sh->bnd_rec;
    std::memcpy(a.slot[0].bnd_off, sh->bnd_off, sizeof(a.slot[0].bnd_off));
    a.slot[0].rhs_out = R.ring + i * slab;
    a.k_end = K;
    HIPCHK(launch_step(m->ref.N, a, m->stream));
  }
  int64_t lb[kMaxLevels + 1];
  fill_level_begin(h, lb);
  HIPCHK(launch_replay_history(Np, R.ring, R.ring + slab, R.ring + 2 * slab, sh->S.ring, K, h.L, lb, m->stream));
  sh->S.tau = 0;
  if ((s = trace_init(sh, sh->S))) return s;
  if ((s = zero_field(sh, R))) return s;
  return begin_replay_segment(sh, 0);
}

static dgrtm_status begin_adjoint(dgrtm_shot sh) {
  dgrtm_mesh m = sh->mesh;
  dgrtm_status s;
  HIPCHK(launch_fill_f64(sh->img, (int64_t)m->ref.Np * m->hm.Ktot, 0.0, m->stream));
  if (sh->replay) return begin_replay_adjoint(sh);
  if ((s = zero_field(sh, sh->R))) return s;
  return begin_segment(sh, (sh->n_global - 1) / sh->C);
}

// work before a global step of the shot's current phase
static dgrtm_status pre_global(dgrtm_shot sh) {
  if (sh->ph != DGRTM_PHASE_FORWARD) return DGRTM_OK;
  if (sh->replay) {
    const int64_t i = sh->n_global - 1 - sh->g;   // the state at global time g = NG - 1 - i
    if (i == 0 || i == 1) {
      dgrtm_mesh m = sh->mesh;
      HIPCHK(hipMemcpyAsync(sh->qsave[i], sh->S.q, (size_t)state_row(m->ref.Np) * m->hm.Ktot * 4,
                            hipMemcpyDeviceToDevice, m->stream));
    }
    return DGRTM_OK;
  }
  if (sh->g % sh->C == 0) return ckpt_copy(sh, sh->S, sh->g / sh->C, true);
  return DGRTM_OK;
}

// boundary traces of the source field after its forward launch at local step tau
static dgrtm_status record_boundary(dgrtm_shot sh, int64_t tau) {
  dgrtm_mesh m = sh->mesh;
  const HostMesh &h = m->hm;
  BndRecArgs r;
  std::memset(&r, 0, sizeof(r));
  r.tr = sh->S.tr;
  r.bface = m->bface;
  r.rec = sh->bnd_rec;
  for (int l = 0; l < kMaxLevels; ++l) {
    r.bnd_off[l] = sh->bnd_off[l];
    r.bnd_cnt[l] = m->bnd_cnt[l];
    r.bnd_begin[l] = m->bnd_begin[l];
  }
  // the levels updated at tau are the finest ones down to the coarsest l with tau on its grid;
  // their faces come first in the list
  int lmin = h.L;
  for (int l = 1; l <= h.L; ++l)
    if ((tau & (((int64_t)1 << (h.L - l)) - 1)) == 0) {
      lmin = l;
      break;
    }
  for (int l = lmin; l <= h.L; ++l) r.n_active += m->bnd_cnt[l - 1];
  r.Ktot = h.Ktot;
  r.L = h.L;
  fill_level_begin(h, r.lev_begin);
  r.tau = tau;
  HIPCHK(launch_bnd_record(m->ref.N, r, m->stream));
  return DGRTM_OK;
}

// work after a global step: recording, phase transitions
static dgrtm_status post_global(dgrtm_shot sh) {
  dgrtm_status s;
  switch (sh->ph) {
    case DGRTM_PHASE_FORWARD:
      sh->g += 1;
      if ((s = record(sh, sh->S, sh->g))) return s;
      if (sh->g == sh->n_global) {
        sh->forward_done = true;
        sh->ph = DGRTM_PHASE_IDLE;
        if (sh->full_rtm) return begin_adjoint(sh);
      }
      return DGRTM_OK;
    case DGRTM_PHASE_RECOMPUTE:
      sh->g += 1;
      if (sh->g == sh->g1) sh->ph = DGRTM_PHASE_BACKWARD;
      return DGRTM_OK;
    case DGRTM_PHASE_BACKWARD:
      if (sh->replay) {   // next backward global step, down to the start of the image window
        if (sh->c + 1 < sh->n_global - sh->g_image_start) return begin_replay_segment(sh, sh->c + 1);
        sh->ph = DGRTM_PHASE_DONE;
        return DGRTM_OK;
      }
      sh->gr += 1;
      if (sh->gr == sh->gr_end) {
        if (sh->c - 1 >= sh->g_image_start / sh->C && sh->c > 0) return begin_segment(sh, sh->c - 1);
        sh->ph = DGRTM_PHASE_DONE;
      }
      return DGRTM_OK;
    default:
      return DGRTM_OK;
  }
}

static bool stepping(const dgrtm_shot sh) {
  return sh->ph == DGRTM_PHASE_FORWARD || sh->ph == DGRTM_PHASE_RECOMPUTE || sh->ph == DGRTM_PHASE_BACKWARD;
}

// one global step of every stepping shot; shots of one mesh at the same mode share launches
static dgrtm_status global_step_shots(dgrtm_shot *shots, int n) {
  dgrtm_status s;
  std::vector<dgrtm_shot> act;
  for (int i = 0; i < n; ++i)
    if (stepping(shots[i])) act.push_back(shots[i]);
  if (act.empty()) return DGRTM_OK;
  dgrtm_mesh m = act[0]->mesh;
  const int nl = act[0]->n_local;
  for (auto *sh : act)
    if ((s = pre_global(sh))) return s;
  std::vector<int> modes(act.size());
  std::vector<bool> rev(act.size());
  std::vector<Field *> fld(act.size());
  for (int ln = 0; ln < nl; ++ln) {
    for (int md : {(int)MODE_PLAIN, (int)MODE_RECORD_SEG, (int)MODE_REPLAY_SEG, (int)MODE_IMAGE})
      for (int prec = 0; prec < 2; ++prec) {
        std::vector<size_t> grp;
        for (size_t i = 0; i < act.size(); ++i) {
          int mode;
          bool r;
          Field *f;
          (void)phase_slot(act[i], mode, r, f);
          if (mode == md && act[i]->args.precision == prec) grp.push_back(i);
        }
        for (size_t b = 0; b < grp.size(); b += kMaxSlots) {
          const size_t e = std::min(grp.size(), b + kMaxSlots);
          int mode;
          bool r;
          Field *f;
          dgrtm_shot first = act[grp[b]];
          (void)phase_slot(first, mode, r, f);
          StepArgs a = mesh_args(m, prec, mode, r, nl);
          a.nslots = (int)(e - b);
          for (size_t i = b; i < e; ++i) {
            dgrtm_shot sh = act[grp[i]];
            a.slot[i - b] = phase_slot(sh, mode, r, f);
            // physical local step of a backward run's rhs (data and source samples)
            if (mode == MODE_IMAGE || mode == MODE_REPLAY_SEG) a.slot[i - b].data_j = sh->n_global * nl - f->tau;
            fld[grp[i]] = f;
          }
          if ((s = launch_slots(first, a, ln))) return s;
          for (size_t i = b; i < e; ++i) {
            dgrtm_shot sh = act[grp[i]];
            if (sh->replay && sh->ph == DGRTM_PHASE_FORWARD)
              if ((s = record_boundary(sh, fld[grp[i]]->tau))) return s;
          }
          for (size_t i = b; i < e; ++i) fld[grp[i]]->tau += 1;
        }
      }
  }
  for (auto *sh : act)
    if ((s = post_global(sh))) return s;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_forward(dgrtm_shot sh, float *traces_out) {
  if (!sh) return fail(DGRTM_ERR_ARG, "dgrtm_forward: bad argument");
  dgrtm_mesh m = sh->mesh;
  dgrtm_status s;
  sh->full_rtm = false;
  if ((s = begin_forward(sh))) return s;
  while (sh->ph == DGRTM_PHASE_FORWARD)
    if ((s = global_step_shots(&sh, 1))) return s;
  if (traces_out && sh->rec.n)
    HIPCHK(hipMemcpyAsync(traces_out, sh->traces, sh->rec.n * (sh->n_global + 1) * 4, hipMemcpyDeviceToDevice,
                          m->stream));
  return DGRTM_OK;
}

static dgrtm_status set_adjoint_params(dgrtm_shot sh, const float *data, int condition, const double *up,
                                       int64_t g_image_start) {
  if (!up) return fail(DGRTM_ERR_ARG, "adjoint: up vector missing");
  const bool trap = (condition & DGRTM_IMAGE_TRAPEZOID) != 0;
  condition &= ~DGRTM_IMAGE_TRAPEZOID;
  if (condition != DGRTM_IMAGE_PRESSURE && condition != DGRTM_IMAGE_CHARACTERISTIC)
    return fail(DGRTM_ERR_ARG, "adjoint: bad condition");
  sh->trapezoid = trap;
  if (g_image_start < 0 || g_image_start >= sh->n_global) return fail(DGRTM_ERR_ARG, "adjoint: bad g_image_start");
  sh->data = data;
  sh->condition = condition;
  for (int i = 0; i < 3; ++i) sh->up[i] = (float)up[i];
  sh->g_image_start = g_image_start;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_adjoint(dgrtm_shot sh, const float *data, int condition, const double *up,
                                      int64_t g_image_start) {
  if (!sh || (sh->rec.n && !data)) return fail(DGRTM_ERR_ARG, "dgrtm_adjoint: bad argument");
  if (!sh->forward_done) return fail(DGRTM_ERR_ARG, "dgrtm_adjoint: run dgrtm_forward first");
  dgrtm_status s;
  if ((s = set_adjoint_params(sh, data, condition, up, g_image_start))) return s;
  if ((s = begin_adjoint(sh))) return s;
  while (sh->ph != DGRTM_PHASE_DONE)
    if ((s = global_step_shots(&sh, 1))) return s;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_shot_begin(dgrtm_shot sh, const float *data, int condition, const double *up,
                                         int64_t g_image_start) {
  if (!sh) return fail(DGRTM_ERR_ARG, "dgrtm_shot_begin: bad argument");
  dgrtm_status s;
  if ((s = set_adjoint_params(sh, data, condition, up, g_image_start))) return s;
  sh->full_rtm = true;
  return begin_forward(sh);
}

extern "C" dgrtm_status dgrtm_step_shots(dgrtm_shot *shots, int n, int64_t n_global) {
  if (!shots || n < 0 || n_global < 0) return fail(DGRTM_ERR_ARG, "dgrtm_step_shots: bad argument");
  for (int i = 0; i < n; ++i) {
    if (!shots[i]) return fail(DGRTM_ERR_ARG, "dgrtm_step_shots: null shot");
    if (shots[i]->mesh != shots[0]->mesh) return fail(DGRTM_ERR_ARG, "dgrtm_step_shots: shots on different meshes");
  }
  dgrtm_status s;
  for (int64_t k = 0; k < n_global; ++k)
    if ((s = global_step_shots(shots, n))) return s;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_shot_traces(dgrtm_shot sh, float *out) {
  if (!sh || !out) return fail(DGRTM_ERR_ARG, "dgrtm_shot_traces: bad argument");
  if (sh->rec.n)
    HIPCHK(hipMemcpyAsync(out, sh->traces, sh->rec.n * (sh->n_global + 1) * 4, hipMemcpyDeviceToDevice,
                          sh->mesh->stream));
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_shot_state(dgrtm_shot sh, int *phase, int64_t *steps_done, int64_t *steps_total) {
  if (!sh) return fail(DGRTM_ERR_ARG, "dgrtm_shot_state: bad argument");
  const int64_t NG = sh->n_global, C = sh->C;
  if (sh->replay) {   // forward NG, then per backward global step: source, then receiver field
    const int64_t total = NG + 2 * (NG - sh->g_image_start);
    int64_t done = 0;
    switch (sh->ph) {
      case DGRTM_PHASE_FORWARD: done = sh->g; break;
      case DGRTM_PHASE_IDLE: done = sh->forward_done ? NG : 0; break;
      case DGRTM_PHASE_DONE: done = total; break;
      default: done = NG + 2 * sh->c + (sh->ph == DGRTM_PHASE_BACKWARD ? 1 : 0);
    }
    if (phase) *phase = sh->ph;
    if (steps_done) *steps_done = done;
    if (steps_total) *steps_total = total;
    return DGRTM_OK;
  }
  // forward NG, then per segment (recompute + backward)
  int64_t total = NG, done = 0;
  for (int64_t c = (NG - 1) / C; c >= sh->g_image_start / C; --c) {
    const int64_t g0 = c * C, g1 = std::min(NG, g0 + C);
    total += (g1 - g0) + (g1 - std::max(g0, sh->g_image_start));
  }
  switch (sh->ph) {
    case DGRTM_PHASE_FORWARD: done = sh->g; break;
    case DGRTM_PHASE_IDLE: done = sh->forward_done ? NG : 0; break;
    case DGRTM_PHASE_DONE: done = total; break;
    default: {
      done = NG;
      for (int64_t c = (NG - 1) / C; c > sh->c; --c) {
        const int64_t g0 = c * C, g1 = std::min(NG, g0 + C);
        done += (g1 - g0) + (g1 - std::max(g0, sh->g_image_start));
      }
      done += (sh->g - sh->g0) + (sh->gr - (NG - sh->g1));
    }
  }
  if (phase) *phase = sh->ph;
  if (steps_done) *steps_done = done;
  if (steps_total) *steps_total = total;
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_image(dgrtm_shot sh, double *image_out, int accumulate) {
  if (!sh || !image_out) return fail(DGRTM_ERR_ARG, "dgrtm_image: bad argument");
  dgrtm_mesh m = sh->mesh;
  HIPCHK(launch_image_to_user(m->ref.Np, sh->img, image_out, m->s2u, m->hm.Ktot, accumulate, m->stream));
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_residual(dgrtm_shot sh, const float *a, const float *b, int64_t n, double *out) {
  if (!sh || !a || !b || !out || n < 0) return fail(DGRTM_ERR_ARG, "dgrtm_residual: bad argument");
  dgrtm_mesh m = sh->mesh;
  HIPCHK(launch_fill_f64(sh->red, 1, 0.0, m->stream));
  HIPCHK(launch_residual(a, b, n, sh->red, m->stream));
  HIPCHK(hipMemcpyAsync(out, sh->red, 8, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return DGRTM_OK;
}

// ------------------------------------------------------------------------------------------------
// test hooks
// ------------------------------------------------------------------------------------------------
extern "C" dgrtm_status dgrtm_apply_rhs(dgrtm_shot sh, const float *q, float *rhs, int reversed) {
  if (!sh || !q || !rhs) return fail(DGRTM_ERR_ARG, "dgrtm_apply_rhs: bad argument");
  dgrtm_mesh m = sh->mesh;
  const int Np = m->ref.Np;
  const int64_t K = m->hm.Ktot;
  dgrtm_status s;
  if ((s = zero_field(sh, sh->S))) return s;
  HIPCHK(launch_to_device_layout(Np, 4, q, sh->S.q, m->s2u, K, m->stream));
  if ((s = trace_init(sh, sh->S))) return s;
  StepArgs a = mesh_args(m, sh->args.precision, MODE_RHS_ONLY, reversed != 0, sh->n_local);
  a.nslots = 1;
  a.slot[0] = field_slot(sh, sh->S);
  a.slot[0].rhs_out = sh->S.ring;
  a.slot[0].tau = 0;
  a.k_end = K;
  HIPCHK(launch_step(m->ref.N, a, m->stream));
  HIPCHK(launch_to_user_layout(Np, 4, sh->S.ring, rhs, m->s2u, K, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_set_state(dgrtm_shot sh, int which, const float *q, const float *h1, const float *h2) {
  if (!sh || (which != 0 && which != 1)) return fail(DGRTM_ERR_ARG, "dgrtm_set_state: bad argument");
  dgrtm_mesh m = sh->mesh;
  const int Np = m->ref.Np;
  const int64_t K = m->hm.Ktot, slab = (int64_t)state_row(Np) * K;
  Field &f = which ? sh->R : sh->S;
  dgrtm_status s;
  if ((s = zero_field(sh, f))) return s;
  if (q) HIPCHK(launch_to_device_layout(Np, 4, q, f.q, m->s2u, K, m->stream));
  // at tau = 0 every element is at own step 0: r(-dt) lives in slot 2, r(-2 dt) in slot 1
  if (h1) HIPCHK(launch_to_device_layout(Np, 4, h1, f.ring + 2 * slab, m->s2u, K, m->stream));
  if (h2) HIPCHK(launch_to_device_layout(Np, 4, h2, f.ring + 1 * slab, m->s2u, K, m->stream));
  if ((s = trace_init(sh, f))) return s;
  HIPCHK(hipStreamSynchronize(m->stream));
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_get_state(dgrtm_shot sh, int which, float *q) {
  if (!sh || !q || (which != 0 && which != 1)) return fail(DGRTM_ERR_ARG, "dgrtm_get_state: bad argument");
  dgrtm_mesh m = sh->mesh;
  Field &f = which ? sh->R : sh->S;
  HIPCHK(launch_to_user_layout(m->ref.Np, 4, f.q, q, m->s2u, m->hm.Ktot, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return DGRTM_OK;
}

extern "C" dgrtm_status dgrtm_run(dgrtm_shot sh, int which, int64_t n_global, int reversed, int with_source) {
  if (!sh || n_global < 0 || (which != 0 && which != 1)) return fail(DGRTM_ERR_ARG, "dgrtm_run: bad argument");
  dgrtm_mesh m = sh->mesh;
  Field &f = which ? sh->R : sh->S;
  StepArgs a = mesh_args(m, sh->args.precision, MODE_PLAIN, reversed != 0, sh->n_local);
  a.nslots = 1;
  a.slot[0] = field_slot(sh, f);
  if (with_source && which == 0 && sh->args.has_source) {
    with_points(a.slot[0], sh->src, 0);
    a.slot[0].wavelet = sh->wavelet;
    if (f.tau + n_global * sh->n_local > sh->n_global * sh->n_local)
      return fail(DGRTM_ERR_ARG, "dgrtm_run: source signal shorter than the run");
  }
  dgrtm_status s;
  for (int64_t g = 0; g < n_global; ++g)
    for (int n = 0; n < sh->n_local; ++n) {
      a.slot[0].tau = f.tau;
      if ((s = launch_slots(sh, a, f.tau))) return s;
      f.tau += 1;
    }
  HIPCHK(hipStreamSynchronize(m->stream));
  return DGRTM_OK;
}
