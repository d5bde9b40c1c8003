// Launch interface of the gfx950 DG kernels (FP32 state, FP64 image accumulation).
//
// Device layout (elements sorted finest level first, each level's segment padded to a multiple
// of 64 so a wavefront never straddles two levels).  Per-element arrays of R rows are tiled:
// element k's row r is at tix(R, r, k) = ((k / 16) R + r) 16 + k % 16, so a row of a 16-element
// tile is 64 contiguous bytes and a tile's R rows are one contiguous block.
//   q     quad layout, qix()       p, vx, vy, vz
//   ring  [3] x quad layout        AB3 right-hand-side history, slot = own step index mod 3
//   tr    [3][Ktot][4][2][FS]      traces p and n.v: slot 0/1 = own step parity, slot 2 = mid step;
//                                  face f's p run starts at 2 f FS and its n.v run at (2 f + 1) FS,
//                                  FS = Nfp rounded up to 4 (one face's two runs are one 128-byte
//                                  line at N = 4, so a neighbour's read of a face fetches no other)
//   geo   [kGeo rows]              rx ry rz sx sy sz tx ty tz, rho c^2, 1/rho, Z, tau_p[4], tau_v[4]
//   nbr   [4 rows]                 neighbour position, or -(boundary type) on a boundary face
//   ncode [4 rows]                 neighbour face | vertex permutation << 2 | neighbour level << 5
//   img   [Np rows] (FP64)         image
//   eflag [Ktot]                   bit0 real element, bit1 has a finer neighbour, bit2 has sources
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgrtm {

constexpr int kGeo = 20;
constexpr int kMaxLevels = 8;

// MODE_REPLAY_SEG and MODE_RHS_REPLAY are MODE_RECORD_SEG and MODE_RHS_ONLY for the source field
// re-simulated backward in time: every boundary face takes its exterior state from the boundary
// traces recorded by the forward run (SlotArgs::bnd_rec) instead of its boundary condition
enum StepMode : int {
  MODE_PLAIN = 0, MODE_RECORD_SEG = 1, MODE_IMAGE = 2, MODE_RHS_ONLY = 3, MODE_REPLAY_SEG = 4, MODE_RHS_REPLAY = 5
};
__host__ __device__ constexpr int base_mode(int mode) {
  return mode == MODE_REPLAY_SEG ? MODE_RECORD_SEG : (mode == MODE_RHS_REPLAY ? MODE_RHS_ONLY : mode);
}

// image rules (SlotArgs::img_rule): bit 0 the source field runs backward too (boundary-trace
// replay) rather than forward from a checkpoint, bit 1 the trapezoid rule instead of the exact
// integral of the dense outputs
constexpr int IMG_SAME_DIR = 1, IMG_TRAPEZOID = 2;

constexpr int kMaxSlots = 8;

// Quad layout of the state and of each rhs of the ring: field c, node n of element k at
// qix(NK, c, n, k), NK = ceil(Np / 4) node quads per field.  A tile's state is one block of
// 4 NK 64 floats; within it, one node quad of one field is 64 floats, element-major with the quad's
// 4 nodes adjacent.  A lane that owns element e and nodes 4 q .. 4 q + 3 (the MFMA C layout) reads
// them with one 16-byte access, and the 64 lanes reading node 4 c + g of element e for g = 0..3
// (the MFMA B layout) read 256 contiguous bytes.  The padding nodes of the last quad hold zeros.
__host__ __device__ constexpr int node_quads(int Np) { return (Np + 3) / 4; }
__host__ __device__ constexpr int state_row(int Np) { return 16 * node_quads(Np); }   // floats per element
__host__ __device__ constexpr int64_t qix(int NK, int c, int n, int64_t k) {
  return ((((k >> 4) * 4 + c) * NK + (n >> 2)) * 16 + (k & 15)) * 4 + (n & 3);
}

// tiled index of row r of element k in an array with R rows per element
__host__ __device__ constexpr int64_t tix(int64_t R, int64_t r, int64_t k) { return ((k >> 4) * R + r) * 16 + (k & 15); }

// face stride of a trace row: Nfp rounded up to a multiple of 4 floats (16-byte aligned runs)
__host__ __device__ constexpr int trace_face_stride(int Nfp) { return (Nfp + 3) & ~3; }
// floats of one element's trace row (four faces, two components)
__host__ __device__ constexpr int trace_row(int Nfp) { return 8 * trace_face_stride(Nfp); }

// Per-shot ("slot") part of a step launch: several shots on the same mesh, at the same phase of
// their global step, share one launch (blockIdx.y selects the slot).
struct SlotArgs {
  float *q, *ring, *tr;
  float *rhs_out;                     // MODE_RHS_ONLY output [4][Np][Ktot]
  const int *eflag;                   // mesh flags | 4 on elements that hold this shot's points
  // point sources: CSR per element (sorted position)
  const int *src_start;               // [Ktot] first point entry
  const int *src_count;               // [Ktot]
  const int *src_point;               // entries -> point id
  const float *src_w;                 // [n_points][Np] projected-delta weights
  const float *wavelet;               // amp_mode 0: source signal at every local step (at local step
                                      // tau; amp_mode 2: at physical local step data_j, n_t samples)
  const float *data;                  // amp_mode 1: [n_points][n_t] samples at global steps
  float *seg_q, *seg_r;               // segment buffer: per level [C N_l][Np][P_l] and [C N_l + 2][Np][P_l]
  double *img;                        // [Np][Ktot]
  int64_t tau;                        // local steps since the start of this field's run
  int64_t n_t;
  int64_t data_j;                     // physical time of this rhs in local steps (amp_mode 1)
  int64_t C;                          // checkpoint interval (global steps)
  int64_t g0, g1;                     // current segment [g0, g1) in global steps
  int64_t NG;                         // global steps of the run
  int64_t image_from;                 // image only where the source step starts at or after this local step
  float up[3];
  float src_scale;
  int amp_mode;                       // 0 wavelet table, 1 linear data interpolation, 2 wavelet at data_j
  int condition;                      // 0 pressure, 1 characteristic
  int img_rule;                       // IMG_SAME_DIR | IMG_TRAPEZOID bits (MODE_IMAGE)
  // boundary-trace record (replay modes): level l's rows at bnd_rec + bnd_off[l-1], row j b of
  // boundary face b at own step j, 2 FS floats: p, then -n.v (as a neighbour would see it)
  const float *bnd_rec;
  int64_t bnd_off[kMaxLevels];
};

struct StepArgs {
  // mesh
  const float *geo;
  const int *nbr;
  const int *ncode;
  const float *ops;                   // FP32 operator fragments (build_op_fragments)
  const uint32_t *ops_bf16;           // split-BF16 operator fragments (build_op_fragments_bf16)
  const int8_t *nbr_index;            // [4][4][6][Nfp]
  // [kMaxSlots][2] per shot slot: tiles handed out beyond the first two per wavefront, and
  // work-groups finished; zero between launches (the last work-group to finish clears them), so
  // launches that share them must not overlap (one stream per mesh)
  uint32_t *tile_ctr;
  int64_t Ktot;
  int L;                              // number of levels
  int64_t lev_begin[kMaxLevels + 1];  // index l-1 -> first position of level l (finest first)
  int64_t bnd_cnt[kMaxLevels];        // boundary faces of level l (index l-1); ncode of a boundary
                                      // face holds its index among them, -1 on padding elements
  // launch
  int64_t k_end;                      // active prefix (multiple of 64), the same for every slot
  int64_t max_groups;                 // cap on work-groups along x; 0 = none
  double dt_local;
  float tau_sign;                     // +1 forward, -1 backward in time
  float out_sign;                     // +1 forward, -1 backward in time
  int n_local;                        // local steps per global step
  int precision;                      // 0 FP32 MFMA, 1 split-BF16 MFMA
  int mode;                           // StepMode
  int nslots;
  SlotArgs slot[kMaxSlots];
};

hipError_t launch_step(int N, const StepArgs &a, hipStream_t st);
// operator fragments in MFMA lane order from row-major Dr, Ds, Dt (Np x Np) and LIFT (Np x 4Nfp)
void build_op_fragments(int N, const float *Dr, const float *Ds, const float *Dt, const float *LIFT, float *out);
int64_t op_fragment_floats(int N);
// hi/lo bf16 operator fragments for the split-BF16 kernel, built from the FP64 operators
void build_op_fragments_bf16(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT,
                             uint32_t *out);
int64_t op_fragment_bf16_words(int N);

struct TraceInitArgs {
  const float *q;
  float *tr;
  const float *geo;
  const int *eflag;
  int64_t Ktot;
  int L;
  int64_t lev_begin[kMaxLevels + 1];
  int64_t tau;
};
hipError_t launch_trace_init(int N, const TraceInitArgs &a, hipStream_t st);

// receivers: out[r * out_stride] = l_r . p(element of r)
hipError_t launch_record(int N, const float *q, int64_t Ktot, const int64_t *rec_pos, const float *rec_l, int64_t n_rec,
                         float *out, int64_t out_stride, hipStream_t st);
// layout conversion user [K][4][Np] <-> device [4][Np][Ktot]
hipError_t launch_to_device_layout(int Np, int nfield, const float *user, float *dev, const int64_t *sorted_to_user,
                                   int64_t Ktot, hipStream_t st);
hipError_t launch_to_user_layout(int Np, int nfield, const float *dev, float *user, const int64_t *sorted_to_user,
                                 int64_t Ktot, hipStream_t st);
hipError_t launch_image_to_user(int Np, const double *img, double *user, const int64_t *sorted_to_user, int64_t Ktot,
                                int accumulate, hipStream_t st);
// r-_S history entries of the segment buffer from the ring at restore time
struct SegInitArgs {
  const float *ring;
  const float *geo;
  const int *eflag;
  float *seg_r;
  int64_t seg_r_off[kMaxLevels];
  int64_t seg_m0[kMaxLevels];
  int64_t Ktot;
  int L;
  int64_t lev_begin[kMaxLevels + 1];
  float up[3];
  int condition;
  int history_before_start;           // the ring holds history for own steps -1, -2 (backward replay run)
};
hipError_t launch_seg_init(int N, const SegInitArgs &a, hipStream_t st);
// boundary traces of the source field after a forward local step: for the boundary faces of the
// levels updated by the launch at local step tau (a prefix of the face list, finest level first),
// p and -n.v of own step j = tau / 2^(L-l) + 1, from trace slot j mod 2, into row j of the record
struct BndRecArgs {
  const float *tr;
  const int *bface;                   // [n_faces] sorted element position * 4 + face, finest first
  float *rec;
  int64_t bnd_off[kMaxLevels];        // level l's rows at rec + bnd_off[l-1]
  int64_t bnd_cnt[kMaxLevels];
  int64_t bnd_begin[kMaxLevels];      // index in bface of level l's first face
  int64_t n_active;                   // faces of the updated levels
  int64_t Ktot;
  int L;
  int64_t lev_begin[kMaxLevels + 1];
  int64_t tau;
};
hipError_t launch_bnd_record(int N, const BndRecArgs &a, hipStream_t st);
struct ReplayLevels {
  int64_t lev_begin[kMaxLevels + 1];
};
// AB3 history of the backward source run at its start: r(-dt_l) into ring slot 2 and r(-2 dt_l)
// into slot 1, from the quadratic through the reversed-time rhs r0, r1, r2 at the global times
// t_f, t_f - dt_g, t_f - 2 dt_g, evaluated at t_f + dt_l and t_f + 2 dt_l
hipError_t launch_replay_history(int Np, const float *r0, const float *r1, const float *r2, float *ring, int64_t Ktot,
                                 int L, const int64_t *lev_begin, hipStream_t st);
// sum over all entries of (a - b)^2 in FP64 into out[0] (out zeroed by the caller)
hipError_t launch_residual(const float *a, const float *b, int64_t n, double *out, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st);

}  // namespace dgrtm
