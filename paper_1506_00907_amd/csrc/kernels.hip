// gfx950 kernels of the nodal DG solver: fused right-hand side + multi-rate AB3 update per
// local step (with optional source-wavefield recording and FP64 image accumulation), trace
// initialisation, receiver sampling, layout conversion and FP64 reductions.
//
// A wavefront owns a tile of 16 consecutive elements; the operator products of the tile run on
// the matrix cores with the 16 elements as the MFMA N dimension.  All field arrays are node-major
// with the element index fastest, so a tile's share of any node row is 64 contiguous bytes.  The
// reference operators are the same for every element and are staged once per work-group in LDS,
// in the MFMA A-operand lane order.
#include "kernels.hpp"

#include <algorithm>
#include <cstring>

namespace dgrtm {

// ------------------------------------------------------------------------------------------
// compile-time node tables of the order-N reference tetrahedron (same numbering as the host:
// node (i,j,l) has barycentric weights (N-i-j-l, i, j, l), l slowest, i fastest)
// ------------------------------------------------------------------------------------------
template <int N>
struct Tab {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  int fmask[4][Nfp];
  int fidx[Np][4];  // position of node n on face f, -1 if not on it
  constexpr Tab() : fmask{}, fidx{} {
    int lat[Np][4] = {};
    int n = 0;
    for (int l = 0; l <= N; ++l)
      for (int j = 0; j <= N - l; ++j)
        for (int i = 0; i <= N - l - j; ++i) {
          lat[n][0] = N - i - j - l;
          lat[n][1] = i;
          lat[n][2] = j;
          lat[n][3] = l;
          ++n;
        }
    const int opp[4] = {3, 2, 0, 1};
    for (int m = 0; m < Np; ++m)
      for (int f = 0; f < 4; ++f) fidx[m][f] = -1;
    for (int f = 0; f < 4; ++f) {
      int c = 0;
      for (int m = 0; m < Np; ++m)
        if (lat[m][opp[f]] == 0) {
          fmask[f][c] = m;
          fidx[m][f] = c;
          ++c;
        }
    }
  }
};

template <int N>
struct Dims {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int F = 4 * Nfp;
  static constexpr int NR = (Np + 15) / 16;   // 16-row tiles of the operators
  static constexpr int NK = (Np + 3) / 4;     // 4-column chunks of D_j
  static constexpr int FC = (Nfp + 3) / 4;    // 4-column chunks per face of LIFT
  static constexpr int OPS = (3 * NR * NK + NR * 4 * FC) * 64;   // operator fragment floats
  static constexpr int TABW = (4 * 4 * 6 * Nfp + 3) / 4;          // face-node map, in 32-bit words
  static constexpr int FS = trace_face_stride(Nfp);               // trace row: run length,
  static constexpr int TRC = FS;                                  // component stride (p, then n.v),
  static constexpr int TRF = 2 * FS;                              // face stride,
  static constexpr int TRS = 4 * TRF;                             // element stride (floats)
};

// index of field c, node n of tile element e in an LDS copy of a tile's state (quad layout)
template <int N>
__device__ __forceinline__ constexpr int lqix(int c, int n, int e) {
  return ((c * Dims<N>::NK + (n >> 2)) * 16 + e) * 4 + (n & 3);
}

// AB3 weights of the full step and of the half step
constexpr float kA0 = 23.0f / 12.0f, kA1 = -16.0f / 12.0f, kA2 = 5.0f / 12.0f;
constexpr float kB0 = 17.0f / 24.0f, kB1 = -7.0f / 24.0f, kB2 = 2.0f / 24.0f;

// Image weights of one own step, per rule (index IMG_SAME_DIR | IMG_TRAPEZOID): the increment is
// dt qS qR + dt^2 sum_s E_s (qS rR_s + rS_s qR) + dt^3 sum C_{s1 s2} rS_s1 rR_s2, with A_s the
// integral from 0 to th of the Lagrange basis on the time nodes {0, -1, -2}:
//   exact, S forward from t_a and R backward from t_b: E_s = ebar_s = int_0^1 A_s,
//     C = Cmix_{s1 s2} = int_0^1 A_s1(th) A_s2(1 - th);
//   exact, both backward from t_b (boundary-trace replay): E_s = ebar_s, C = int_0^1 A_s1 A_s2
//     (the matrix of the imaging section);
//   trapezoid rule, dt/2 (S R at both ends), the far ends from the AB3 update: E_s = a_s / 2 and
//     C = 0 (mixed direction) or C = a_s1 a_s2 / 2 (both backward)
#define DGRTM_E_EXACT 19.0 / 24.0, -5.0 / 12.0, 1.0 / 8.0
#define DGRTM_E_TRAP 23.0 / 24.0, -16.0 / 24.0, 5.0 / 24.0
__constant__ double kImgW[4][12] = {
    {DGRTM_E_EXACT, 3341.0 / 10080.0, -667.0 / 5040.0, 43.0 / 1120.0, -667.0 / 5040.0, 19.0 / 420.0, -13.0 / 1008.0,
     43.0 / 1120.0, -13.0 / 1008.0, 37.0 / 10080.0},
    {DGRTM_E_EXACT, 4703.0 / 5040.0, -457.0 / 840.0, 52.0 / 315.0, -457.0 / 840.0, 103.0 / 315.0, -251.0 / 2520.0,
     52.0 / 315.0, -251.0 / 2520.0, 17.0 / 560.0},
    {DGRTM_E_TRAP, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {DGRTM_E_TRAP, 529.0 / 288.0, -368.0 / 288.0, 115.0 / 288.0, -368.0 / 288.0, 256.0 / 288.0, -80.0 / 288.0,
     115.0 / 288.0, -80.0 / 288.0, 25.0 / 288.0}};
#undef DGRTM_E_EXACT
#undef DGRTM_E_TRAP

// own-step index of the source-field record that an image step at receiver own step m reads
__device__ __forceinline__ int64_t image_source_step(const SlotArgs &sl, int lev, int64_t m) {
  return (sl.img_rule & IMG_SAME_DIR) ? m : (sl.NG << (lev - 1)) - m - 1;
}

// where a replayed boundary face's record row is: face b (its index among the boundary faces of
// level lev), for an element at own step m of the backward run (physical own step NG 2^(lev-1) - m)
template <int N>
__device__ __forceinline__ const float *replay_row(const StepArgs &a, const SlotArgs &sl, int lev, int64_t m, int b) {
  const int64_t j = (sl.NG << (lev - 1)) - m;
  return sl.bnd_rec + sl.bnd_off[lev - 1] + (j * a.bnd_cnt[lev - 1] + b) * (2 * Dims<N>::FS);
}

// Copy nwords 32-bit words from global to LDS with the whole work-group: all 16-byte loads of a
// thread are issued before its LDS stores, so the copy costs one memory latency.
__device__ __forceinline__ int level_of(const int64_t *lev_begin, int L, int64_t k) {
  // segments are stored finest first, so starts decrease with the level number
  for (int l = 1; l < L; ++l)
    if (k >= lev_begin[l - 1]) return l;
  return L;
}

__device__ __forceinline__ int64_t level_end(const int64_t *lev_begin, int L, int l) {
  return l == 1 ? lev_begin[L] : lev_begin[l - 2];
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// select one of four compile-time constants by the lane group g = lane / 16
__device__ __forceinline__ int sel4(int g, int a, int b, int c, int d) {
  return g == 0 ? a : (g == 1 ? b : (g == 2 ? c : d));
}

// round-to-nearest-even bf16 of x (upper 16 bits of the FP32 pattern)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// x = hi + lo + O(2^-17 |x|), hi and lo bf16
__device__ __forceinline__ void split_bf16(float x, short &hi, short &lo) {
  const uint32_t h = bf16_bits(x);
  hi = (short)h;
  lo = (short)bf16_bits(x - __uint_as_float(h << 16));
}

// Geometry of face f of the lane's element and where its neighbour's traces live.
struct FaceCtx {
  float nx, ny, nz, Fs, taup, tauv;
  int nb, f2;
  int rep_b;   // replay modes: the face's index among its level's boundary faces, else -1
  const float *trp;
  const int8_t *tab;
};

// face f of element k: normal, J_f/J, penalty parameters, and where the neighbour's traces are
// (nb, code: the face's neighbour entry and code)
template <int N>
__device__ __forceinline__ FaceCtx face_ctx_of(const StepArgs &a, const SlotArgs &sl, int f, const float *gg, int nb,
                                               int code) {
  constexpr int Nfp = Dims<N>::Nfp;
  const int64_t K = a.Ktot;
  FaceCtx c;
  float nx, ny, nz;
  if (f == 0) { nx = -gg[6]; ny = -gg[7]; nz = -gg[8]; }
  else if (f == 1) { nx = -gg[3]; ny = -gg[4]; nz = -gg[5]; }
  else if (f == 2) { nx = gg[0] + gg[3] + gg[6]; ny = gg[1] + gg[4] + gg[7]; nz = gg[2] + gg[5] + gg[8]; }
  else { nx = -gg[0]; ny = -gg[1]; nz = -gg[2]; }
  c.Fs = sqrtf(nx * nx + ny * ny + nz * nz);  // J_f / J
  const float inv = 1.0f / c.Fs;
  c.nx = nx * inv; c.ny = ny * inv; c.nz = nz * inv;
  c.nb = nb;
  c.taup = a.tau_sign * gg[12 + f];
  c.tauv = a.tau_sign * gg[16 + f];
  c.trp = sl.tr;
  c.tab = a.nbr_index;
  c.f2 = 0;
  c.rep_b = (nb < 0 && code >= 0) ? code : -1;
  if (c.nb >= 0) {
    c.f2 = code & 3;
    const int perm = (code >> 2) & 7;
    const int shn = a.L - (code >> 5);
    // neighbour on its own step grid -> parity slot, otherwise (one level coarser) its mid step
    const int slot = ((sl.tau & ((1LL << shn) - 1)) == 0) ? (int)((sl.tau >> shn) & 1) : 2;
    c.trp = sl.tr + (int64_t)slot * Dims<N>::TRS * K;
    c.tab = a.nbr_index + ((f * 4 + c.f2) * 6 + perm) * Nfp;
  }
  return c;
}

// Everything after the operator products, in the MFMA C layout (lane: element e, rows
// 16 rt + 4 g + i): point sources, output of a bare rhs, AB3 update, rhs ring, traces of the new
// state and of the half step, source-wavefield segment record and FP64 image accumulation.
// offsets of level `lev` in a slot's segment buffer (levels stored finest first, like the elements)
__device__ __forceinline__ void seg_offsets(const StepArgs &a, int64_t C, int Np, int lev, int64_t &oq, int64_t &orr) {
  oq = 0;
  orr = 0;
  for (int l = 1; l < lev; ++l) {
    const int64_t P = level_end(a.lev_begin, a.L, l) - a.lev_begin[l - 1];
    const int64_t nst = C << (l - 1);
    oq += nst * Np * P;
    orr += (nst + 2) * Np * P;
  }
}

// QLDS: the old state comes from an LDS tile in the quad layout (field c, node n of element e at
// lqix(c, n, e)) instead of global memory; HLDS: the two older rhs come from LDS tiles (sh1, sh2).
// TR2 (needs both): no per-lane stores of the state, the rhs or the traces; the new state replaces
// the first older rhs in sh1, the new rhs the second in sh2 and the half-step state the old state in
// sq, for tile_traces and the block stores to write out with 16-byte stores (the old state's tile
// is then the first to be free for the next tile's copies).
// PRE (image step): the tile's segment rows are in LDS at sseg and the image values at the lane's
// nodes in imv_pre, both loaded before the update.
// TRQ (needs QLDS, not TR2): the new state also replaces the old one in sq, for tile_traces to write
// the own-step traces from; only the half-step traces are written here, per lane.
// Without HLDS / TR2 the older rhs are read, and the new rhs and state written, as one 16-byte
// access per field and node quad.
template <int N, int MODE, bool QLDS = false, bool HLDS = false, bool TR2 = false, bool PRE = false,
          bool TRQ = false, bool PF = false>
__device__ __forceinline__ void tile_tail(const StepArgs &a, const SlotArgs &sl, int64_t k, int g, int lev, int sh,
                                          int64_t m, int flag, float *sq, int e,
                                          float Z, const float (&nfx)[4], const float (&nfy)[4], const float (&nfz)[4],
                                          v4f (&rp)[Dims<N>::NR], v4f (&rvx)[Dims<N>::NR], v4f (&rvy)[Dims<N>::NR],
                                          v4f (&rvz)[Dims<N>::NR], float *sh1 = nullptr,
                                          float *sh2 = nullptr, const float *sseg = nullptr,
                                          const double *imv_pre = nullptr) {
  constexpr Tab<N> T{};
  constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, F = Dims<N>::F, NR = Dims<N>::NR;
  const int64_t K = a.Ktot;
  constexpr int NQ4 = node_quads(Np);
  const bool valid = (flag & 1) != 0;
  if (a.out_sign < 0.0f) {
#pragma unroll
    for (int rt = 0; rt < NR; ++rt) {
      rp[rt] = -rp[rt]; rvx[rt] = -rvx[rt]; rvy[rt] = -rvy[rt]; rvz[rt] = -rvz[rt];
    }
  }
  // ---- point sources (projected delta into the pressure equation)
  if (valid && (flag & 4)) {
    const int s0 = sl.src_start[k], scn = sl.src_count[k];
    for (int en = s0; en < s0 + scn; ++en) {
      const int pt = sl.src_point[en];
      float amp = 0.0f;
      if (sl.amp_mode == 0) {
        amp = sl.wavelet[sl.tau];
      } else if (sl.amp_mode == 2) {
        amp = (sl.data_j >= 0 && sl.data_j < sl.n_t) ? sl.wavelet[sl.data_j] : 0.0f;
      } else {
        const int64_t j = sl.data_j;
        const int64_t gq = j / a.n_local, rem = j % a.n_local;
        if (j >= 0 && (gq < sl.n_t - 1 || (gq == sl.n_t - 1 && rem == 0))) {
          const float *d = sl.data + (int64_t)pt * sl.n_t;
          if (rem == 0) amp = d[gq];
          else {
            const float th = (float)rem / (float)a.n_local;
            amp = (1.0f - th) * d[gq] + th * d[gq + 1];
          }
        }
      }
      amp *= sl.src_scale;
      const float *w = sl.src_w + (int64_t)pt * Np;
#pragma unroll
      for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int n = 16 * rt + 4 * g + i;
          if (16 * rt + 15 < Np || n < Np) rp[rt][i] += amp * w[n];
        }
    }
  }
  if (!valid) {
    if constexpr (TR2) {
      // a padding element keeps its state and passes its history on, as the per-lane path does
#pragma unroll
      for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int n = 16 * rt + 4 * g + i;
          if (!(16 * rt + 15 < Np || n < Np)) continue;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float h = sh1[lqix<N>(c, n, e)];
            sh2[lqix<N>(c, n, e)] = h;
            sh1[lqix<N>(c, n, e)] = sq[lqix<N>(c, n, e)];
          }
        }
    }
    return;
  }
  if constexpr (MODE == MODE_RHS_ONLY) {
#pragma unroll
    for (int rt = 0; rt < NR; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = 16 * rt + 4 * g + i;
        if (16 * rt + 15 < Np || n < Np) {
          sl.rhs_out[qix(NQ4, 0, n, k)] = rp[rt][i];
          sl.rhs_out[qix(NQ4, 1, n, k)] = rvx[rt][i];
          sl.rhs_out[qix(NQ4, 2, n, k)] = rvy[rt][i];
          sl.rhs_out[qix(NQ4, 3, n, k)] = rvz[rt][i];
        }
      }
    return;
  }
  const int64_t slab = (int64_t)state_row(Np) * K;
  const float dtl = (float)(a.dt_local * (double)(1LL << sh));
  float *__restrict__ R0 = sl.ring + (m % 3) * slab;
  const float *__restrict__ R1 = sl.ring + ((m + 2) % 3) * slab;
  const float *__restrict__ R2 = sl.ring + ((m + 1) % 3) * slab;
  constexpr int FS = Dims<N>::FS, TRC = Dims<N>::TRC, TRS = Dims<N>::TRS;
  float *__restrict__ trw = sl.tr + ((m + 1) & 1) * (int64_t)TRS * K;
  float *__restrict__ trm = sl.tr + (int64_t)2 * TRS * K;
  const bool mid = (flag & 2) != 0;
  float *q = sl.q;
  const float ux = sl.up[0], uy = sl.up[1], uz = sl.up[2];
  const float zs = sl.condition ? Z : 0.0f;
  int64_t kk = 0, Pl = 0, jS = 0, oq = 0, orr = 0;
  bool do_img = false;
  if constexpr (MODE == MODE_RECORD_SEG || MODE == MODE_IMAGE) {
    kk = k - a.lev_begin[lev - 1];
    Pl = level_end(a.lev_begin, a.L, lev) - a.lev_begin[lev - 1];
    seg_offsets(a, sl.C, Np, lev, oq, orr);
  }
  if constexpr (MODE == MODE_RECORD_SEG) jS = m - (sl.g0 << (lev - 1));
  if constexpr (MODE == MODE_IMAGE) {
    const int64_t mS = image_source_step(sl, lev, m);   // the source step this receiver step pairs with
    jS = mS - (sl.g0 << (lev - 1));
    do_img = (mS << sh) >= sl.image_from && jS >= 0 && jS < ((sl.g1 - sl.g0) << (lev - 1));
  }
  const double dtd = a.dt_local * (double)(1LL << sh);

  // the rhs history of the lane's node quad in row tile rt (rows past the last quad hold no nodes)
  float4 hq1[NR][4], hq2[NR][4];
  auto load_hist = [&](int rt) {
    const int qd = 4 * rt + g;
    const bool qok = 4 * rt + 3 < NQ4 || qd < NQ4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t iq = qix(NQ4, c, 4 * (qok ? qd : 0), k);
      hq1[rt][c] = *reinterpret_cast<const float4 *>(R1 + iq);
      hq2[rt][c] = *reinterpret_cast<const float4 *>(R2 + iq);
    }
  };
  if constexpr (PF && !HLDS) load_hist(0);
  // Row tile by row tile: every load of the tile (rhs history, q, segment data, image) is issued
  // before any store, so the loads of one row tile are in flight together (stores to the ring could
  // otherwise alias later ring loads and serialise every load behind the previous store).  With PF
  // the next row tile's history loads are issued before this row tile's work, so that their
  // latency overlaps it.
#pragma unroll
  for (int rt = 0; rt < NR; ++rt) {
    float h1[4][4], h2[4][4], qo[4][4];
    float sqv[4] = {0.f, 0.f, 0.f, 0.f}, srv[4][3] = {};
    double imv[4] = {0.0, 0.0, 0.0, 0.0};
    // node quad of this lane's four rows in this row tile (rows past the last quad hold no nodes)
    const int qd = 4 * rt + g;
    const bool qok = 4 * rt + 3 < NQ4 || qd < NQ4;
    if constexpr (!HLDS) {
      if constexpr (PF) {
        __builtin_amdgcn_sched_barrier(0);
        if (rt + 1 < NR) load_hist(rt + 1);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        load_hist(rt);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float4 a1 = hq1[rt][c], a2 = hq2[rt][c];
        h1[0][c] = qok ? a1.x : 0.f; h1[1][c] = qok ? a1.y : 0.f; h1[2][c] = qok ? a1.z : 0.f; h1[3][c] = qok ? a1.w : 0.f;
        h2[0][c] = qok ? a2.x : 0.f; h2[1][c] = qok ? a2.y : 0.f; h2[2][c] = qok ? a2.z : 0.f; h2[3][c] = qok ? a2.w : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = 16 * rt + 4 * g + i;
      const bool ok = (16 * rt + 15 < Np || n < Np);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t idx = qix(NQ4, c, ok ? n : 0, k);
        if constexpr (HLDS) {
          h1[i][c] = sh1[lqix<N>(c, ok ? n : 0, e)];
          h2[i][c] = sh2[lqix<N>(c, ok ? n : 0, e)];
        }
        if constexpr (QLDS) qo[i][c] = sq[lqix<N>(c, ok ? n : 0, e)];
        else qo[i][c] = ok ? q[idx] : 0.f;
      }
    }
    if constexpr (MODE == MODE_IMAGE) {
      if (do_img) {   // uniform over the tile; all loads of the row tile in one batch
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int n = 16 * rt + 4 * g + i;
          const int nn = (16 * rt + 15 < Np || n < Np) ? n : 0;   // (rows past Np are not used)
          if constexpr (PRE) {   // the tile's segment rows, in LDS: [q][r(jS+2)][r(jS+1)][r(jS)] x Np x 16
            sqv[i] = sseg[(0 * Np + nn) * 16 + e];
            srv[i][0] = sseg[(1 * Np + nn) * 16 + e];
            srv[i][1] = sseg[(2 * Np + nn) * 16 + e];
            srv[i][2] = sseg[(3 * Np + nn) * 16 + e];
          } else {
            const float *sqp = sl.seg_q + oq;
            const float *srp = sl.seg_r + orr;
            sqv[i] = sqp[jS * Np * Pl + tix(Np, nn, kk)];
            srv[i][0] = srp[(jS + 2) * Np * Pl + tix(Np, nn, kk)];
            srv[i][1] = srp[(jS + 1) * Np * Pl + tix(Np, nn, kk)];
            srv[i][2] = srp[jS * Np * Pl + tix(Np, nn, kk)];
          }
          if constexpr (PRE) imv[i] = imv_pre[rt * 4 + i];
          else imv[i] = sl.img[tix(Np, nn, k)];
        }
      }
    }
    if constexpr (!TR2) {
      // new rhs and state of the lane's node quad, one 16-byte store per field (rows past Np in
      // an existing quad are padding: zero operator rows and zero history leave them zero)
      if (qok) {
        const v4f rr[4] = {rp[rt], rvx[rt], rvy[rt], rvz[rt]};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t iq = qix(NQ4, c, 4 * qd, k);
          float qq[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) qq[i] = qo[i][c] + dtl * (kA0 * rr[c][i] + kA1 * h1[i][c] + kA2 * h2[i][c]);
          *reinterpret_cast<float4 *>(R0 + iq) = float4{rr[c][0], rr[c][1], rr[c][2], rr[c][3]};
          *reinterpret_cast<float4 *>(q + iq) = float4{qq[0], qq[1], qq[2], qq[3]};
          if constexpr (TRQ) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sq[lqix<N>(c, 4 * qd + i, e)] = qq[i];   // (read above, not again)
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = 16 * rt + 4 * g + i;
      if (!(16 * rt + 15 < Np || n < Np)) continue;
      const float r[4] = {rp[rt][i], rvx[rt][i], rvy[rt][i], rvz[rt][i]};
      float qn[4], qm[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        qn[c] = qo[i][c] + dtl * (kA0 * r[c] + kA1 * h1[i][c] + kA2 * h2[i][c]);
        qm[c] = qo[i][c] + dtl * (kB0 * r[c] + kB1 * h1[i][c] + kB2 * h2[i][c]);
        if constexpr (TR2) {   // (these slots were read above and are not read again)
          sh1[lqix<N>(c, n, e)] = qn[c];
          sh2[lqix<N>(c, n, e)] = r[c];
          sq[lqix<N>(c, n, e)] = qm[c];
        }
      }
      if constexpr (MODE == MODE_RECORD_SEG) {
        const float qminus = qo[i][0] - zs * (ux * qo[i][1] + uy * qo[i][2] + uz * qo[i][3]);
        const float rminus = r[0] - zs * (ux * r[1] + uy * r[2] + uz * r[3]);
        sl.seg_q[oq + jS * Np * Pl + tix(Np, n, kk)] = qminus;
        sl.seg_r[orr + (jS + 2) * Np * Pl + tix(Np, n, kk)] = rminus;
      }
      if constexpr (MODE == MODE_IMAGE) {
        if (do_img) {
          const double qS = sqv[i];
          const double rS[3] = {srv[i][0], srv[i][1], srv[i][2]};
          const double qR = qo[i][0] + zs * (ux * qo[i][1] + uy * qo[i][2] + uz * qo[i][3]);
          const double rR[3] = {r[0] + zs * (ux * r[1] + uy * r[2] + uz * r[3]),
                                h1[i][0] + zs * (ux * h1[i][1] + uy * h1[i][2] + uz * h1[i][3]),
                                h2[i][0] + zs * (ux * h2[i][1] + uy * h2[i][2] + uz * h2[i][3])};
          const double *W = kImgW[sl.img_rule & 3];
          double inc2 = 0.0, inc3 = 0.0;
#pragma unroll
          for (int s = 0; s < 3; ++s) inc2 += W[s] * (qS * rR[s] + rS[s] * qR);
#pragma unroll
          for (int s1 = 0; s1 < 3; ++s1)
#pragma unroll
            for (int s2 = 0; s2 < 3; ++s2) inc3 += W[3 + 3 * s1 + s2] * rS[s1] * rR[s2];
          sl.img[tix(Np, n, k)] = imv[i] + dtd * (qS * qR + dtd * (inc2 + dtd * inc3));
        }
      }
      if constexpr (TR2) continue;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const int fi = sel4(g, T.fidx[min(16 * rt + i, Np - 1)][f], T.fidx[min(16 * rt + 4 + i, Np - 1)][f],
                            T.fidx[min(16 * rt + 8 + i, Np - 1)][f], T.fidx[min(16 * rt + 12 + i, Np - 1)][f]);
        if (fi >= 0) {
          const int64_t r0 = (int64_t)k * TRS + f * Dims<N>::TRF + fi;
          const int64_t r1 = r0 + TRC;
          if constexpr (!TRQ) {
            trw[r0] = qn[0];
            trw[r1] = nfx[f] * qn[1] + nfy[f] * qn[2] + nfz[f] * qn[3];
          }
          if (mid) {
            trm[r0] = qm[0];
            trm[r1] = nfx[f] * qm[1] + nfy[f] * qm[2] + nfz[f] * qm[3];
          }
        }
      }
    }
  }
}

// Traces of the new state (and of the half step, for elements with a finer neighbour) from the
// LDS tiles left by tile_tail<..., TR2>: lane (e, g) writes face g of element e, one 16-byte store
// per 4 face nodes (the face runs are 16-byte aligned; the padding after the last node is written
// with zeros and never read).
template <int N, bool MID = true>
__device__ __forceinline__ void tile_traces(const StepArgs &a, const SlotArgs &sl, int64_t k, int g, int e, int64_t m,
                                            int flag, const float *sq, const float *sqm, const float (&nfx)[4],
                                            const float (&nfy)[4], const float (&nfz)[4]) {
  constexpr Tab<N> T{};
  constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, FS = Dims<N>::FS, TRC = Dims<N>::TRC, TRS = Dims<N>::TRS;
  if (!(flag & 1)) return;
  const int64_t K = a.Ktot;
  const bool mid = (flag & 2) != 0;
  const float nx = g == 0 ? nfx[0] : (g == 1 ? nfx[1] : (g == 2 ? nfx[2] : nfx[3]));
  const float ny = g == 0 ? nfy[0] : (g == 1 ? nfy[1] : (g == 2 ? nfy[2] : nfy[3]));
  const float nz = g == 0 ? nfz[0] : (g == 1 ? nfz[1] : (g == 2 ? nfz[2] : nfz[3]));
  float *trw = sl.tr + ((m + 1) & 1) * (int64_t)TRS * K + k * TRS + g * Dims<N>::TRF;
  float *trm = sl.tr + (int64_t)2 * TRS * K + k * TRS + g * Dims<N>::TRF;
#pragma unroll
  for (int j = 0; j < FS / 4; ++j) {
    float p[4], v[4], pm[4], vm[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = 4 * j + u;
      p[u] = v[u] = pm[u] = vm[u] = 0.0f;
      if (s < Nfp) {
        const int node = sel4(g, T.fmask[0][s], T.fmask[1][s], T.fmask[2][s], T.fmask[3][s]);
        p[u] = sq[lqix<N>(0, node, e)];
        v[u] = nx * sq[lqix<N>(1, node, e)] + ny * sq[lqix<N>(2, node, e)] + nz * sq[lqix<N>(3, node, e)];
        if constexpr (MID) {
          pm[u] = sqm[lqix<N>(0, node, e)];
          vm[u] = nx * sqm[lqix<N>(1, node, e)] + ny * sqm[lqix<N>(2, node, e)] + nz * sqm[lqix<N>(3, node, e)];
        }
      }
    }
    *reinterpret_cast<float4 *>(trw + 4 * j) = float4{p[0], p[1], p[2], p[3]};
    *reinterpret_cast<float4 *>(trw + TRC + 4 * j) = float4{v[0], v[1], v[2], v[3]};
    if (MID && mid) {
      *reinterpret_cast<float4 *>(trm + 4 * j) = float4{pm[0], pm[1], pm[2], pm[3]};
      *reinterpret_cast<float4 *>(trm + TRC + 4 * j) = float4{vm[0], vm[1], vm[2], vm[3]};
    }
  }
}

// converts the volume accumulators (sum_j D_j U_j and D_j p) into the pressure and velocity rhs
template <int NR>
__device__ __forceinline__ void volume_to_rhs(const float *gg, const v4f (&cp)[NR], const v4f (&w0)[NR],
                                              const v4f (&w1)[NR], const v4f (&w2)[NR], v4f (&rp)[NR],
                                              v4f (&rvx)[NR], v4f (&rvy)[NR], v4f (&rvz)[NR]) {
  const float rx = gg[0], ry = gg[1], rz = gg[2], sx = gg[3], sy = gg[4], sz = gg[5], tx = gg[6], ty = gg[7],
              tz = gg[8], rc2 = gg[9], irho = gg[10];
#pragma unroll
  for (int rt = 0; rt < NR; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float wr = w0[rt][i], ws = w1[rt][i], wt = w2[rt][i];
      rp[rt][i] = -rc2 * cp[rt][i];
      rvx[rt][i] = -irho * (rx * wr + sx * ws + tx * wt);
      rvy[rt][i] = -irho * (ry * wr + sy * ws + ty * wt);
      rvz[rt][i] = -irho * (rz * wr + sz * ws + tz * wt);
    }
}

// ------------------------------------------------------------------------------------------
// The step kernel for N <= 4 (FP32 or split-BF16 products).  One wavefront owns a tile of 16
// consecutive elements.  The element-batched operator products run on the matrix cores: FP32 on
// v_mfma_f32_16x16x4_f32 with A = 16 operator rows x 4 columns (lane l holds A[l%16][l/16]),
// B = 4 input nodes x 16 elements (lane l holds B[l/16][l%16]), C = 16 rows x 16 elements (lane
// l holds rows 4(l/16)+i, i=0..3, of element l%16); split-BF16 on v_mfma_f32_16x16x16_bf16 with
// 16-column chunks.  All elementwise work (geometric factors, penalties, AB3, traces, image) runs
// in the C layout: lane l handles the element e = l%16 and, in row tile rt, the nodes
// n = 16 rt + 4 (l/16) + i.  The kernel is pipelined across tiles:
//  - The volume operator fragments live in registers for the whole kernel (81 per lane at N = 4
//    in FP32, 108 in split-BF16; the matrix cores read their A operand from there) and the LIFT
//    fragments and the face-node map in LDS (13.4 KB), which leaves room for the data tiles.
//  - Everything a tile reads in bulk is copied HBM -> LDS by global_load_lds (no registers hold
//    data in flight): its state, geometry and the two older rhs as 1 KB blocks, and the
//    neighbours' face runs as 16-byte copies (the node permutation is applied when reading).
//  - A tile's copies go out early: its state (and, in the image step, geometry and neighbour
//    runs) at the end of the previous tile, before that tile's block stores; in the forward and
//    recompute steps its geometry and neighbour runs right after the previous tile's surface
//    terms; its history at its own top, landing while the operator products run.
//  - Launches with at least three tiles per wavefront stagger the starts of a work-group's
//    wavefronts by about a quarter tile and hand tiles out from a counter.
// The copies are issued from inline assembly and every wait on them is explicit: vmcnt counts
// vector-memory instructions (loads and stores) in issue order, so "at most n outstanding" means
// everything but the last n issued has landed.  The compiler's own waits cover only the loads it
// can see (element ids and flags, source data), which makes them at worst stricter in hardware,
// never weaker.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
  return (uint32_t)(size_t)((__attribute__((address_space(3))) const void *)p);
}
// 16 bytes per lane to LDS at lds + 16 lane (lds wave-uniform)
__device__ __forceinline__ void lds_copy16(const void *g, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g),
               "s"(__builtin_amdgcn_readfirstlane(lds))
               : "memory", "m0");
}
#define DGRTM_WAIT_VM(n) asm volatile("s_waitcnt vmcnt(" #n ")" ::: "memory")
// at most n vector-memory instructions outstanding (n a compile-time count)
template <int n>
__device__ __forceinline__ void wait_vm_at_most() {
  static_assert(n >= 0 && n <= 63, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(n) : "memory");
}

// one tile's block of ROWS rows x 16 floats (contiguous, 16-byte aligned) -> LDS, 1 KB per copy
template <int ROWS>
__device__ __forceinline__ void copy_block(const float *src, uint32_t lds, int lane) {
#pragma unroll
  for (int j = 0; j < (ROWS + 15) / 16; ++j)
    if (ROWS % 16 == 0 || 16 * j + (lane >> 2) < ROWS) lds_copy16(src + 256 * j + 4 * lane, lds + 1024 * j);
}

// LDS -> one tile's block of ROWS rows x 16 floats, 16-byte stores
template <int ROWS>
__device__ __forceinline__ void store_block(const float *lds, float *dst, int lane) {
#pragma unroll
  for (int j = 0; j < (ROWS + 15) / 16; ++j)
    if (ROWS % 16 == 0 || 16 * j + (lane >> 2) < ROWS)
      *reinterpret_cast<float4 *>(dst + 256 * j + 4 * lane) = *reinterpret_cast<const float4 *>(lds + 256 * j + 4 * lane);
}

// NBYTES (a multiple of 16) from global to LDS by LDS copies, 1 KB per wavefront instruction, the
// work-group's four wavefronts taking alternate kilobytes
template <int NBYTES>
__device__ __forceinline__ void stage_dma(const void *src, void *dst, int wave, int lane) {
  static_assert(NBYTES % 16 == 0, "16-byte copies");
  constexpr int NCH = (NBYTES + 1023) / 1024;
#pragma unroll
  for (int c = 0; c < NCH; ++c)
    if ((c & 3) == wave && c * 1024 + 16 * lane < NBYTES)
      lds_copy16(reinterpret_cast<const char *>(src) + c * 1024 + 16 * lane, lds_addr(dst) + c * 1024);
}

// C += A_hi B_hi + A_hi B_lo + A_lo B_hi (A: uint4 fragment with hi in x, y and lo in z, w)
#define DGRTM_MF3(A, BH, BL, C)                                                                          \
  do {                                                                                                   \
    const v4s ah_ = __builtin_bit_cast(v4s, uint2{(A).x, (A).y});                                        \
    const v4s al_ = __builtin_bit_cast(v4s, uint2{(A).z, (A).w});                                        \
    C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah_, BH, C, 0, 0, 0);                                  \
    C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah_, BL, C, 0, 0, 0);                                  \
    C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al_, BH, C, 0, 0, 0);                                  \
  } while (0)

// Split-BF16 form: every operator product A x is evaluated as A_hi x_hi + A_hi x_lo + A_lo x_hi
// on v_mfma_f32_16x16x16_bf16 with FP32 accumulation (A = A_hi + A_lo and x = x_hi + x_lo in
// bf16).  Lane l holds A[l%16][4(l/16)..4(l/16)+3] and B[4(l/16)..+3][l%16]; C as above.
// Operator fragments: per (operator, row tile, 16-column chunk) 64 lanes x (4 hi + 4 lo) bf16.
template <int N>
struct DimsB {
  static constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, NR = Dims<N>::NR;
  static constexpr int NK = (Np + 15) / 16;    // 16-column chunks of D_j
  static constexpr int FC = (Nfp + 15) / 16;   // 16-column chunks per face of LIFT
  static constexpr int FRAG = 3 * NR * NK + NR * 4 * FC;          // fragments
  static constexpr int OPS_U4 = FRAG * 64;                        // uint4 per fragment lane
};

template <int N>
struct DmaDims {
  static constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, FC = Dims<N>::FC;
  static constexpr int QW = 4 * Dims<N>::NK * 64;    // floats of one tile's state (quad layout)
  static constexpr int GW = kGeo * 16;               // geometry tile
  static constexpr int FS = Dims<N>::FS;
  static constexpr int TW = 8 * 16 * FS;             // neighbour face runs [face][p, n.v][FS/4][16][4]
  static constexpr int WAVE = QW + GW + TW + 2 * QW;  // LDS words per wavefront
};

template <int N, int MODE, int PREC>
__global__ __launch_bounds__(256) void step_kernel_dma(const StepArgs a) {
  constexpr Tab<N> T{};
  using Dm = Dims<N>;
  using DD = DmaDims<N>;
  using DB = DimsB<N>;
  constexpr int Np = Dm::Np, Nfp = Dm::Nfp, F = Dm::F, NR = Dm::NR, NK = Dm::NK, FC = Dm::FC;
  constexpr int QW = DD::QW;
  // the replay modes are the record and rhs-only modes with replayed boundary faces
  constexpr bool REPLAY = MODE == MODE_REPLAY_SEG || MODE == MODE_RHS_REPLAY;
  constexpr int BM = base_mode(MODE);
  constexpr bool HIST = BM != MODE_RHS_ONLY;
  // LIFT fragments: FP32 [NR][4 FC][64] floats, or split-BF16 [NR][4 FC_B][64] x (4 hi + 4 lo) bf16
  constexpr int SLW = PREC ? NR * 4 * DB::FC * 64 * 4 : NR * 4 * FC * 64;
  __shared__ __align__(16) uint32_t stabw[Dm::TABW];
  __shared__ __align__(16) float sL[SLW];
  __shared__ __align__(16) float stile[4][DD::WAVE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = lane & 15, g = lane >> 4;
  const int8_t *stab = reinterpret_cast<const int8_t *>(stabw);
  const int64_t K = a.Ktot;
  const int64_t ntiles = a.k_end >> 4;
  const SlotArgs &sl = a.slot[blockIdx.y];
  // Tiles.  Wavefront w of work-group b takes tiles 4 b + w and then 4 b + w + W (W wavefronts in
  // the grid).  A launch with at least 3 W tiles hands out the rest in order from the slot's
  // counter, and its wavefronts start about a quarter of a tile apart, so that their bursts of
  // copies and stores (and those of every other work-group, which run in step) interleave instead
  // of all reaching the memory system at once; the wavefronts that start later take fewer tiles.
  // A smaller launch keeps the stride W throughout and starts at once.
  const int64_t nfirst = 4 * (int64_t)gridDim.x;
  const bool dyn = ntiles >= 3 * nfirst;
  uint32_t *const ctr = a.tile_ctr + 2 * blockIdx.y;
  auto grab = [&]() -> uint32_t {   // the returned value is read only after an explicit wait
    uint32_t v = 0u;
    if (lane == 0) v = atomicAdd(ctr, 1u);
    return v;
  };
  int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  const bool live = tile < ntiles;   // (always when dyn, where tile < W <= ntiles)
  float *const q_t = stile[wave];
  float *const g_t = q_t + QW;
  float *const n_t = g_t + DD::GW;
  float *const h_t = n_t + DD::TW;
  const uint32_t lq = __builtin_amdgcn_readfirstlane(lds_addr(q_t));
  const uint32_t lg = lq + 4 * QW, ln = lg + 4 * DD::GW, lh = ln + 4 * DD::TW;

  int nbv[4], codev[4], flag;
  // element ids, codes and flags of a tile (registers; the tile loop reads them only after an
  // explicit wait, so they are marked consumed there and the compiler places no wait of its own)
  auto load_elem = [&](int64_t t, int (&nb)[4], int (&cd)[4], int &fl) {
    const int64_t kk = t * 16 + e;
    fl = sl.eflag[kk];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      nb[f] = a.nbr[tix(4, f, kk)];
      cd[f] = a.ncode[tix(4, f, kk)];
    }
  };
  // a tile's state
  auto issue_q = [&](int64_t t) { copy_block<16 * NK>(sl.q + t * QW, lq, lane); };
  // a tile's geometry
  auto issue_g = [&](int64_t t) { copy_block<kGeo>(a.geo + tix(kGeo, 0, t * 16), lg, lane); };
  // a tile's neighbours' face runs (nb, cd: the tile's neighbour ids and codes)
  auto issue_t = [&](int64_t t, const int (&nbs)[4], const int (&cds)[4]) {
    int lev_t = 0;
    int64_t m_t = 0;
    if constexpr (REPLAY) {
      lev_t = level_of(a.lev_begin, a.L, t * 16);
      m_t = sl.tau >> (a.L - lev_t);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int nb = nbs[f], code = cds[f];
      const int f2 = code & 3, perm = (code >> 2) & 7, shn = a.L - (code >> 5);
      const int slot = nb >= 0 ? (((sl.tau & ((1LL << shn) - 1)) == 0) ? (int)((sl.tau >> shn) & 1) : 2) : 0;
      const float *trp = sl.tr + (int64_t)slot * Dm::TRS * K;
      // a replayed boundary face: its recorded run, in the element's own node order
      const bool rep = REPLAY && nb < 0 && code >= 0;
      // lane (g, e) copies nodes 4g .. 4g+3 of the neighbour's face run (in the neighbour's node
      // order) to [face][component][g][e][4]; the surface terms apply the node permutation
      if ((nb >= 0 || rep) && 4 * g < Dm::FS) {
        const float *run, *run2;
        if (rep) {
          run = replay_row<N>(a, sl, lev_t, m_t, code) + 4 * g;
          run2 = run + Dm::FS;
        } else {
          run = trp + (int64_t)nb * Dm::TRS + f2 * Dm::TRF + 4 * g;
          run2 = run + Dm::TRC;
        }
        lds_copy16(run, ln + 4 * (2 * f + 0) * 16 * Dm::FS);
        lds_copy16(run2, ln + 4 * (2 * f + 1) * 16 * Dm::FS);
      }
      (void)perm;
    }
  };
  auto issue_gt = [&](int64_t t, const int (&nbs)[4], const int (&cds)[4]) {
    issue_g(t);
    issue_t(t, nbs, cds);
  };
  // the two older rhs of a tile: issued once the tile's fields have landed, so that they travel
  // while the tile's operator products run instead of in the same burst as the fields
  auto issue_hist = [&](int64_t t) {
    const int64_t k0 = t * 16;
    const int lev = level_of(a.lev_begin, a.L, k0);
    const int64_t m = sl.tau >> (a.L - lev);
    const int64_t slab = (int64_t)state_row(Np) * K;
    copy_block<16 * NK>(sl.ring + ((m + 2) % 3) * slab + (k0 >> 4) * QW, lh, lane);
    copy_block<16 * NK>(sl.ring + ((m + 1) % 3) * slab + (k0 >> 4) * QW, lh + 4 * QW, lane);
  };
  // the first tile's state, geometry and element data travel while the operators are staged
  if (live) {
    issue_q(tile);
    issue_g(tile);
    load_elem(tile, nbv, codev, flag);
  }
  // volume operator fragments -> registers (A operands of every volume product of every tile)
  float fD[3][NR][NK];          // FP32
  uint4 fDb[3][NR][DB::NK];     // split-BF16: hi in (x, y), lo in (z, w)
  if constexpr (PREC == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int c = 0; c < NK; ++c) fD[j][rt][c] = a.ops[((j * NR + rt) * NK + c) * 64 + lane];
    stage_dma<4 * SLW>(a.ops + 3 * NR * NK * 64, sL, wave, lane);
  } else {
    const uint4 *ob = reinterpret_cast<const uint4 *>(a.ops_bf16);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int c = 0; c < DB::NK; ++c) fDb[j][rt][c] = ob[((j * NR + rt) * DB::NK + c) * 64 + lane];
    stage_dma<4 * SLW>(ob + 3 * NR * DB::NK * 64, sL, wave, lane);
  }
  stage_dma<4 * Dm::TABW>(a.nbr_index, stabw, wave, lane);
  // all of the above has landed (a builtin wait, so that the compiler places no wait for the
  // operator registers inside the tile loop, where it would also wait for the tile copies)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (!live) return;
#pragma unroll
  for (int f = 0; f < 4; ++f) asm volatile("" : "+v"(nbv[f]), "+v"(codev[f]));
  asm volatile("" : "+v"(flag));
  issue_t(tile, nbv, codev);
  if (dyn)
    for (int i = 0; i < wave; ++i) __builtin_amdgcn_s_sleep(127);
  DGRTM_WAIT_VM(0);
  int64_t nxt = tile + nfirst;

  // Order of a tile's vector-memory traffic (vmcnt counts loads and stores in issue order):
  //   top      wait until at most SW are outstanding: the previous tile's SW block stores may still
  //            run, everything issued before them (this tile's copies) has landed; issue the history
  //   surface  (forward and recompute) the next tile's geometry and neighbour runs, into tiles that
  //            this tile no longer reads
  //   end      traces of the new state; the next tile's state (and, for the image step, geometry
  //            and neighbour runs); then the SW block stores of the new state and the new rhs
  constexpr bool EARLY_GT = HIST && BM != MODE_IMAGE;
  constexpr int SW = HIST ? 2 * NK : 0;   // 16 NK rows per block store: NK instructions each

  while (true) {
    // this tile's state, geometry and neighbour runs have landed, and every LDS read of the
    // previous tile is done
    __builtin_amdgcn_sched_barrier(0);
    wait_vm_at_most<SW>();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (HIST) issue_hist(tile);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t k = tile * 16 + e;
    int nbn[4], coden[4], flagn = 0;
    uint32_t vnn = 0u;
    if (nxt < ntiles) {   // both land while this tile computes
      if (dyn) vnn = grab();
      load_elem(nxt, nbn, coden, flagn);
    }
    const int lev = level_of(a.lev_begin, a.L, tile * 16);   // uniform over the tile
    const int sh = a.L - lev;
    const int64_t m = sl.tau >> sh;

    float gg[kGeo];
#pragma unroll
    for (int i = 0; i < kGeo; ++i) gg[i] = g_t[i * 16 + e];
    const float rx = gg[0], ry = gg[1], rz = gg[2], sx = gg[3], sy = gg[4], sz = gg[5], tx = gg[6], ty = gg[7],
                tz = gg[8];
    const float rc2 = gg[9], irho = gg[10];

    // ---- volume: Cp = sum_j D_j U_j and W_j = D_j p
    v4f cp[NR], w0[NR], w1[NR], w2[NR];
#pragma unroll
    for (int rt = 0; rt < NR; ++rt) cp[rt] = w0[rt] = w1[rt] = w2[rt] = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == 0) {
#pragma unroll
      for (int c = 0; c < NK; ++c) {
        const int mm = 4 * c + g;
        const bool ok = 4 * c + 3 < Np || mm < Np;
        const int mr = ok ? mm : 0;
        const float p = ok ? q_t[lqix<N>(0, mr, e)] : 0.f;
        const float vx = ok ? q_t[lqix<N>(1, mr, e)] : 0.f;
        const float vy = ok ? q_t[lqix<N>(2, mr, e)] : 0.f;
        const float vz = ok ? q_t[lqix<N>(3, mr, e)] : 0.f;
        const float Ur = rx * vx + ry * vy + rz * vz;
        const float Us = sx * vx + sy * vy + sz * vz;
        const float Ut = tx * vx + ty * vy + tz * vz;
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) {
          cp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fD[0][rt][c], Ur, cp[rt], 0, 0, 0);
          w0[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fD[0][rt][c], p, w0[rt], 0, 0, 0);
          cp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fD[1][rt][c], Us, cp[rt], 0, 0, 0);
          w1[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fD[1][rt][c], p, w1[rt], 0, 0, 0);
          cp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fD[2][rt][c], Ut, cp[rt], 0, 0, 0);
          w2[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fD[2][rt][c], p, w2[rt], 0, 0, 0);
        }
      }
    } else {
      // lane (e, g) supplies B rows 16 c + 4 g .. + 3: node quad 4 c + g of each field, one
      // 16-byte LDS read each (quads past the last hold no nodes and give zeros)
#pragma unroll
      for (int c = 0; c < DB::NK; ++c) {
        const int qd = 4 * c + g;
        const bool ok = 4 * c + 3 < NK || qd < NK;
        const int qr = ok ? qd : 0;
        float4 p4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(0, 4 * qr, e)]);
        float4 x4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(1, 4 * qr, e)]);
        float4 y4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(2, 4 * qr, e)]);
        float4 z4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(3, 4 * qr, e)]);
        if (!ok) p4 = x4 = y4 = z4 = float4{0.f, 0.f, 0.f, 0.f};
        const float pv[4] = {p4.x, p4.y, p4.z, p4.w}, xv[4] = {x4.x, x4.y, x4.z, x4.w};
        const float yv[4] = {y4.x, y4.y, y4.z, y4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
        v4s urh, url, ush, usl, uth, utl, ph, pl;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          short h, l;
          split_bf16(rx * xv[v] + ry * yv[v] + rz * zv[v], h, l); urh[v] = h; url[v] = l;
          split_bf16(sx * xv[v] + sy * yv[v] + sz * zv[v], h, l); ush[v] = h; usl[v] = l;
          split_bf16(tx * xv[v] + ty * yv[v] + tz * zv[v], h, l); uth[v] = h; utl[v] = l;
          split_bf16(pv[v], h, l); ph[v] = h; pl[v] = l;
        }
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) {
          const uint4 ar = fDb[0][rt][c], as = fDb[1][rt][c], at = fDb[2][rt][c];
          DGRTM_MF3(ar, urh, url, cp[rt]);
          DGRTM_MF3(as, ush, usl, cp[rt]);
          DGRTM_MF3(at, uth, utl, cp[rt]);
          DGRTM_MF3(ar, ph, pl, w0[rt]);
          DGRTM_MF3(as, ph, pl, w1[rt]);
          DGRTM_MF3(at, ph, pl, w2[rt]);
        }
      }
    }
    v4f rp[NR], rvx[NR], rvy[NR], rvz[NR];
    volume_to_rhs<NR>(gg, cp, w0, w1, w2, rp, rvx, rvy, rvz);

    // ---- surface: rp -= LIFT Pp (accumulated by the MFMA with -Pp), G_f = LIFT_f Pv, rv -= n_f G_f
    float nfx[4], nfy[4], nfz[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      float nx, ny, nz;
      if (f == 0) { nx = -tx; ny = -ty; nz = -tz; }
      else if (f == 1) { nx = -sx; ny = -sy; nz = -sz; }
      else if (f == 2) { nx = rx + sx + tx; ny = ry + sy + ty; nz = rz + sz + tz; }
      else { nx = -rx; ny = -ry; nz = -rz; }
      const float Fs = sqrtf(nx * nx + ny * ny + nz * nz);  // J_f / J
      const float inv = 1.0f / Fs;
      nx *= inv; ny *= inv; nz *= inv;
      nfx[f] = nx; nfy[f] = ny; nfz[f] = nz;
      const int nb = nbv[f];
      const float taup = a.tau_sign * gg[12 + f], tauv = a.tau_sign * gg[16 + f];
      // exterior state without branches: p+ = cP p- + p_nb and (n-.v)+ = -(cP (n-.v)- + (n_nb.v)_nb),
      // with p_nb, (n.v)_nb the neighbour's traces on an interior face and 0 on a boundary face;
      // cP = 1 on a rigid wall, -1 on a free surface, 0 on a transparent or interior face
      const bool inner = nb >= 0;
      // a replayed boundary face takes its whole exterior state from the record
      const bool rep = REPLAY && !inner && codev[f] >= 0;
      const float cP = REPLAY ? 0.0f : (nb == -1 ? 1.0f : (nb == -3 ? -1.0f : 0.0f));
      const int f2 = inner ? (codev[f] & 3) : 0, perm = inner ? ((codev[f] >> 2) & 7) : 0;
      v4f G[NR];
#pragma unroll
      for (int rt = 0; rt < NR; ++rt) G[rt] = v4f{0.f, 0.f, 0.f, 0.f};
      // the penalty terms at face node s (volume node `node`; zero unless sv: s exists)
      auto pen = [&](int s, int node, bool sv, float &mPp, float &Pv) {
        const float pm = q_t[lqix<N>(0, node, e)];
        const float nvm = nx * q_t[lqix<N>(1, node, e)] + ny * q_t[lqix<N>(2, node, e)] + nz * q_t[lqix<N>(3, node, e)];
        // the neighbour's node matching face node s of this face
        const int t = rep ? min(s, Nfp - 1) : stab[((f * 4 + f2) * 6 + perm) * Nfp + min(s, Nfp - 1)];
        const int toff = (t >> 2) * 64 + e * 4 + (t & 3);
        const float tp = (inner || rep) ? n_t[(2 * f + 0) * 16 * Dm::FS + toff] : 0.0f;
        const float tv = (inner || rep) ? n_t[(2 * f + 1) * 16 * Dm::FS + toff] : 0.0f;
        const float pp = cP * pm + tp;
        const float nvp = -(cP * nvm + tv);
        const float dp = pp - pm, dnv = nvp - nvm;
        mPp = sv ? -0.5f * rc2 * (dnv - taup * dp) * Fs : 0.0f;
        Pv = sv ? 0.5f * irho * (dp - tauv * dnv) * Fs : 0.0f;
      };
      if constexpr (PREC == 0) {
#pragma unroll
        for (int cc = 0; cc < FC; ++cc) {   // lane (e, g) takes face node 4 cc + g
          const bool sv = 4 * cc + 3 < Nfp || 4 * cc + g < Nfp;
          const int node = sel4(g, T.fmask[f][4 * cc], T.fmask[f][min(4 * cc + 1, Nfp - 1)],
                                T.fmask[f][min(4 * cc + 2, Nfp - 1)], T.fmask[f][min(4 * cc + 3, Nfp - 1)]);
          float mPp, Pv;
          pen(4 * cc + g, node, sv, mPp, Pv);
#pragma unroll
          for (int rt = 0; rt < NR; ++rt) {
            const float al = sL[(rt * 4 * FC + f * FC + cc) * 64 + lane];
            rp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(al, mPp, rp[rt], 0, 0, 0);
            G[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(al, Pv, G[rt], 0, 0, 0);
          }
        }
      } else {
        const uint4 *sLb = reinterpret_cast<const uint4 *>(sL);
#pragma unroll
        for (int cc = 0; cc < DB::FC; ++cc) {   // lane (e, g) takes face nodes 16 cc + 4 g + v
          v4s pph, ppl, pvh, pvl;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int s = 16 * cc + 4 * g + v;
            const bool sv = 16 * cc + 12 + v < Nfp || s < Nfp;
            const int node = sel4(g, T.fmask[f][min(16 * cc + v, Nfp - 1)], T.fmask[f][min(16 * cc + 4 + v, Nfp - 1)],
                                  T.fmask[f][min(16 * cc + 8 + v, Nfp - 1)], T.fmask[f][min(16 * cc + 12 + v, Nfp - 1)]);
            float mPp, Pv;
            pen(s, node, sv, mPp, Pv);
            short h, l;
            split_bf16(mPp, h, l); pph[v] = h; ppl[v] = l;
            split_bf16(Pv, h, l); pvh[v] = h; pvl[v] = l;
          }
#pragma unroll
          for (int rt = 0; rt < NR; ++rt) {
            const uint4 al = sLb[(rt * 4 * DB::FC + f * DB::FC + cc) * 64 + lane];
            DGRTM_MF3(al, pph, ppl, rp[rt]);
            DGRTM_MF3(al, pvh, pvl, G[rt]);
          }
        }
      }
#pragma unroll
      for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          rvx[rt][i] -= nx * G[rt][i];
          rvy[rt][i] -= ny * G[rt][i];
          rvz[rt][i] -= nz * G[rt][i];
        }
    }
    const float *sseg = nullptr;
    double imv[NR * 4];   // the image at this lane's nodes (image step), loaded with the segment rows
    if constexpr (BM == MODE_IMAGE) {
      // the source-wavefield segment rows this receiver step correlates with go to the geometry
      // and neighbour-trace tiles, which the tile no longer reads
      static_assert(4 * Np * 16 <= DD::GW + DD::TW, "segment rows fit in the geometry and trace tiles");
      const int64_t mS = image_source_step(sl, lev, m);
      const int64_t jS = mS - (sl.g0 << (lev - 1));
      if ((mS << sh) >= sl.image_from && jS >= 0 && jS < ((sl.g1 - sl.g0) << (lev - 1))) {
        int64_t oq, orr;
        seg_offsets(a, sl.C, Np, lev, oq, orr);
        const int64_t Pl = level_end(a.lev_begin, a.L, lev) - a.lev_begin[lev - 1];
        const int64_t kk0 = tile * 16 - a.lev_begin[lev - 1];
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the surface terms' LDS reads are done
        copy_block<Np>(sl.seg_q + oq + jS * Np * Pl + tix(Np, 0, kk0), lg, lane);
        copy_block<Np>(sl.seg_r + orr + (jS + 2) * Np * Pl + tix(Np, 0, kk0), lg + 4 * Np * 16, lane);
        copy_block<Np>(sl.seg_r + orr + (jS + 1) * Np * Pl + tix(Np, 0, kk0), lg + 8 * Np * 16, lane);
        copy_block<Np>(sl.seg_r + orr + jS * Np * Pl + tix(Np, 0, kk0), lg + 12 * Np * 16, lane);
        sseg = g_t;
#pragma unroll
        for (int rt = 0; rt < NR; ++rt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int n = 16 * rt + 4 * g + i;
            imv[rt * 4 + i] = sl.img[tix(Np, (16 * rt + 15 < Np || n < Np) ? n : 0, k)];   // (rows past Np unused)
          }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    DGRTM_WAIT_VM(0);   // the history copies (and the next tile's element data) have landed
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int f = 0; f < 4; ++f) asm volatile("" : "+v"(nbn[f]), "+v"(coden[f]));
    asm volatile("" : "+v"(flagn), "+v"(vnn));
    // the tile after the next
    const int64_t nn = dyn ? 2 * nfirst + __builtin_amdgcn_readfirstlane(vnn) : nxt + nfirst;
    const bool more = nxt < ntiles;
    if constexpr (EARLY_GT) {
      // the geometry tile was read at the top and the neighbour runs by the surface terms
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      if (more) issue_gt(nxt, nbn, coden);
      __builtin_amdgcn_sched_barrier(0);
    }
    tile_tail<N, BM, true, HIST, HIST, BM == MODE_IMAGE>(a, sl, k, g, lev, sh, m, flag, q_t, e, gg[11], nfx, nfy,
                                                        nfz, rp, rvx, rvy, rvz, h_t, h_t + QW, sseg,
                                                        BM == MODE_IMAGE ? imv : nullptr);
    if constexpr (HIST) {
      tile_traces<N>(a, sl, k, g, e, m, flag, h_t, q_t, nfx, nfy, nfz);
      // the old-state tile (half-step state by now) and, for the image step, the segment rows in
      // the geometry and neighbour tiles have been read
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      if (more) {
        issue_q(nxt);
        if constexpr (!EARLY_GT) issue_gt(nxt, nbn, coden);
      }
      __builtin_amdgcn_sched_barrier(0);
      // new state and new rhs of the tile: element-contiguous rows, 16 bytes per lane
      const int64_t k0 = tile * 16;
      store_block<16 * NK>(h_t, sl.q + (k0 >> 4) * QW, lane);
      store_block<16 * NK>(h_t + QW, sl.ring + (m % 3) * ((int64_t)state_row(Np) * K) + (k0 >> 4) * QW, lane);
    } else {
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      if (more) {
        issue_q(nxt);
        issue_gt(nxt, nbn, coden);
      }
    }
    if (!more) break;
    tile = nxt;
    nxt = nn;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      nbv[f] = nbn[f];
      codev[f] = coden[f];
    }
    flag = flagn;
  }
  if (dyn) {
    // the last work-group to finish clears the counters for the next launch (every wavefront of a
    // dyn launch reaches this point)
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t done = atomicAdd(ctr + 1, 1u);
      if (done + 1u == gridDim.x) {
        ctr[0] = 0u;
        ctr[1] = 0u;
      }
    }
  }
}

// The step kernel for N >= 5 (FP32 or split-BF16 products), with the tile mapping and MFMA
// layout of step_kernel_dma.  Its operators (in LDS when they fit, else read through the caches)
// leave room in LDS for one tile per wavefront, but not for the neighbour runs and the history:
// each wavefront's state and geometry tiles come by LDS copies, issued for the next tile as soon
// as the update has read the state; neighbour traces and the older rhs are read per lane.
// OPS_LDS: where the operator fragments are read from: 0 through the caches, 1 all of them from LDS,
// 2 the lift fragments from LDS and the volume fragments through the caches
template <int N, int MODE, int OPS_LDS, int PREC>
__global__ __launch_bounds__(256) void step_kernel_lowreg(const StepArgs a) {
  constexpr Tab<N> T{};
  using Dm = Dims<N>;
  using DD = DmaDims<N>;
  using DB = DimsB<N>;
  constexpr int Np = Dm::Np, Nfp = Dm::Nfp, NR = Dm::NR, NK = Dm::NK, FC = Dm::FC;
  // operator fragment floats: FP32 [3][NR][NK][64] + [NR][4 FC][64], split-BF16 the same in uint4
  constexpr int OPSW = PREC ? DB::OPS_U4 * 4 : Dm::OPS;
  constexpr int QW = DD::QW, GW = DD::GW;
  // the replay modes are the record and rhs-only modes with replayed boundary faces
  constexpr bool REPLAY = MODE == MODE_REPLAY_SEG || MODE == MODE_RHS_REPLAY;
  constexpr int BM = base_mode(MODE);
  // volume chunks per unrolled loop step where a chunk's fragments are read in its own step
  // (N = 6 has no registers to spare for two)
  constexpr int VU = N >= 6 ? 1 : 2;
  // floats of the volume fragments, and of the operators held in LDS
  constexpr int DW = PREC ? 3 * NR * DB::NK * 64 * 4 : 3 * NR * NK * 64;
  constexpr int LDSOPS = OPS_LDS == 1 ? OPSW : (OPS_LDS == 2 ? OPSW - DW : 0);
  extern __shared__ __align__(16) float sdyn[];   // [operators in LDS][4 wavefronts][QW + GW]
  __shared__ __align__(16) uint32_t stabw[Dm::TABW];   // face-node map [4][4][6][Nfp]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = lane & 15, g_lane = lane >> 4;
  const int64_t K = a.Ktot;
  const int64_t ntiles = a.k_end >> 4;
  const SlotArgs &sl = a.slot[blockIdx.y];
  float *const q_t = sdyn + LDSOPS + wave * (QW + GW);
  float *const g_t = q_t + QW;
  const uint32_t lq = __builtin_amdgcn_readfirstlane(lds_addr(q_t));
  const uint32_t lg = lq + 4 * QW;
  // Tiles as in step_kernel_dma: two fixed tiles per wavefront, then (a launch with at least three
  // tiles per wavefront) tiles handed out by the slot's counter and staggered wavefront starts
  const int64_t nfirst = 4 * (int64_t)gridDim.x;
  const bool dyn = ntiles >= 3 * nfirst;
  uint32_t *const ctr = a.tile_ctr + 2 * blockIdx.y;
  int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  auto issue = [&](int64_t t) {
    copy_block<16 * NK>(sl.q + t * QW, lq, lane);
    copy_block<kGeo>(a.geo + tix(kGeo, 0, t * 16), lg, lane);
  };
  if (tile < ntiles) issue(tile);
  // neighbour entries and codes of a tile's faces: with the operators in LDS they are loaded with
  // the tile's copies (the face contexts need them before the volume terms), else at its top
  int nbv[4], cdv[4];
  auto load_nb = [&](int64_t t) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      nbv[f] = a.nbr[tix(4, f, t * 16 + e)];
      cdv[f] = a.ncode[tix(4, f, t * 16 + e)];
    }
  };
  if constexpr (OPS_LDS == 1) {
    if (tile < ntiles) load_nb(tile);
  }
  const float *ops = PREC ? reinterpret_cast<const float *>(a.ops_bf16) : a.ops;
  const float *lift = ops + DW;
  if constexpr (OPS_LDS == 1) {
    stage_dma<4 * OPSW>(ops, sdyn, wave, lane);
    ops = sdyn;
    lift = sdyn + DW;
  } else if constexpr (OPS_LDS == 2) {
    stage_dma<4 * (OPSW - DW)>(lift, sdyn, wave, lane);
    lift = sdyn;
  }
  stage_dma<4 * Dm::TABW>(a.nbr_index, stabw, wave, lane);
  const int8_t *stab = reinterpret_cast<const int8_t *>(stabw);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (dyn)
    for (int i = 0; i < wave; ++i) __builtin_amdgcn_s_sleep(127);
  int64_t nxt = tile + nfirst;

  while (tile < ntiles) {
    // this tile's state and geometry have landed
    __builtin_amdgcn_sched_barrier(0);
    DGRTM_WAIT_VM(0);
    __builtin_amdgcn_sched_barrier(0);
    // An opaque zero keeps the operator-fragment reads inside the tile loop (hoisting them out would
    // pin every fragment in registers for the whole kernel).  At N = 6, outside the FP32 forward
    // step, it also keeps there the lane's face-node and node-quad selections, which depend on its
    // row group g: hoisted, they would hold about a hundred registers through the loop, which the
    // update's history prefetch and the split-BF16 form's second fragment buffer need instead;
    // recomputed, they cost a few hundred VALU instructions per tile.
    int opaque0;
    asm volatile("s_mov_b32 %0, 0" : "=s"(opaque0));
    const int g = (N >= 6 && (BM != MODE_PLAIN || PREC == 1)) ? g_lane + opaque0 : g_lane;
    const int64_t k = tile * 16 + e;
    uint32_t vnn = 0u;   // the tile after the next (counter value), read at the end of this tile
    if (dyn && nxt < ntiles && lane == 0) vnn = atomicAdd(ctr, 1u);
    if constexpr (OPS_LDS != 1) load_nb(tile);   // (they land while the volume terms run)
    const float *__restrict__ fD = ops + opaque0;                       // [3][NR][NK][64]
    const float *__restrict__ fL = lift + opaque0;                      // [NR][4*FC][64]
    const uint4 *__restrict__ bD = reinterpret_cast<const uint4 *>(ops) + opaque0;          // split-BF16
    const uint4 *__restrict__ bL = reinterpret_cast<const uint4 *>(lift) + opaque0;
    const int flag = sl.eflag[k];
    const int lev = level_of(a.lev_begin, a.L, tile * 16);   // uniform over the tile
    const int sh = a.L - lev;
    const int64_t m = sl.tau >> sh;

    float gg[kGeo];
#pragma unroll
    for (int i = 0; i < kGeo; ++i) gg[i] = g_t[i * 16 + e];
    const float rx = gg[0], ry = gg[1], rz = gg[2], sx = gg[3], sy = gg[4], sz = gg[5], tx = gg[6], ty = gg[7],
                tz = gg[8];
    const float rc2 = gg[9], irho = gg[10];

    // The faces' contexts and their neighbour traces (all faces' in one batch, in both forms).
    // With the operators in LDS they come before the volume terms, which then wait on no global
    // load, so the gathers land while they run; with the volume fragments read through the caches
    // they come after (a gather issued before would be waited for by the first fragment wait).
    float nfx[4], nfy[4], nfz[4];
    FaceCtx fcs[4];
    // FP32: lane (e, g) takes face node 4 cc + g; split-BF16: face nodes 16 cc + 4 g + v
    constexpr int TPN = PREC ? DB::FC * 4 : FC;
    float tpa[4][TPN], tva[4][TPN];
    auto faces = [&]() {
#pragma unroll
      for (int f = 0; f < 4; ++f) fcs[f] = face_ctx_of<N>(a, sl, f, gg, nbv[f], cdv[f]);
      // the neighbour's traces at face node s of face fc
      auto nbnode = [&](const FaceCtx &fc, int s, float &p_, float &v_) {
        const bool inner = fc.nb >= 0;
        const int sidx = min(s, Nfp - 1);
        // the face-node map in LDS: fc.tab points into the global copy at the same offset
        const int8_t *tab = stab + (fc.tab - a.nbr_index);
        const float *nbt = fc.trp + (int64_t)(inner ? fc.nb : 0) * Dm::TRS + fc.f2 * Dm::TRF + tab[inner ? sidx : 0];
        p_ = inner ? nbt[0] : 0.0f;
        v_ = inner ? nbt[Dm::TRC] : 0.0f;
        if constexpr (REPLAY) {
          if (fc.rep_b >= 0) {   // a replayed boundary face: the recorded run, own node order
            const float *row = replay_row<N>(a, sl, lev, m, fc.rep_b);
            p_ = row[sidx];
            v_ = row[Dm::FS + sidx];
          }
        }
      };
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < TPN; ++i)
          nbnode(fcs[f], PREC ? 16 * (i >> 2) + 4 * g + (i & 3) : 4 * i + g, tpa[f][i], tva[f][i]);
    };
    if constexpr (OPS_LDS == 1) faces();
    // ---- volume: Cp = sum_j D_j U_j and W_j = D_j p
    v4f cp[NR], w0[NR], w1[NR], w2[NR];
#pragma unroll
    for (int rt = 0; rt < NR; ++rt) cp[rt] = w0[rt] = w1[rt] = w2[rt] = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == 0) {
      // the B operands of one 4-column chunk: node 4 c + g of the lane's element, four fields
      auto bload = [&](int c, float (&b)[4]) {
        const int mm = 4 * c + g;
        const bool ok = mm < Np;
        const int mr = ok ? mm : 0;
#pragma unroll
        for (int f = 0; f < 4; ++f) b[f] = ok ? q_t[lqix<N>(f, mr, e)] : 0.f;
      };
      // the products of one 4-column chunk, its B operands given
      auto vchunkb = [&](const float (&b)[4], const float (&fa)[3][NR]) {
        const float p = b[0], vx = b[1], vy = b[2], vz = b[3];
        const float Ur = rx * vx + ry * vy + rz * vz;
        const float Us = sx * vx + sy * vy + sz * vz;
        const float Ut = tx * vx + ty * vy + tz * vz;
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) {
          cp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0][rt], Ur, cp[rt], 0, 0, 0);
          cp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1][rt], Us, cp[rt], 0, 0, 0);
          cp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[2][rt], Ut, cp[rt], 0, 0, 0);
          w0[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0][rt], p, w0[rt], 0, 0, 0);
          w1[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1][rt], p, w1[rt], 0, 0, 0);
          w2[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[2][rt], p, w2[rt], 0, 0, 0);
        }
      };
      // the products of one 4-column chunk, A fragments given
      auto vchunk = [&](int c, const float (&fa)[3][NR]) {
        float b[4];
        bload(c, b);
        vchunkb(b, fa);
      };
      auto vload = [&](int c, float (&fa)[3][NR]) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int rt = 0; rt < NR; ++rt) fa[j][rt] = fD[((j * NR + rt) * NK + c) * 64 + lane];
      };
      float fa[3][NR];
      if constexpr (OPS_LDS != 1) {
        // Fragments read through the caches, two column chunks per 8-byte load (the paired copy
        // after the lift fragments): two register buffers of chunk pairs, the next pair's loads in
        // flight while a pair's products run.  The loads past the last pair re-read it
        // (unconditional loads keep the waits exact), and scheduling barriers keep each pair's
        // loads in one batch, so that the wait before a pair's products leaves the other buffer's
        // loads in flight.
        static_assert(N >= 6, "the paired volume fragments are built for N >= 6");
        constexpr int NK2 = (NK + 1) / 2;
        const float2 *__restrict__ fP = reinterpret_cast<const float2 *>(a.ops + Dm::OPS) + opaque0;
        // a pair's A fragments and its B operands (from LDS) are loaded together, a pair ahead
        auto pload = [&](int c2, float2 (&fp)[3][NR], float (&b)[2][4]) {
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int rt = 0; rt < NR; ++rt) fp[j][rt] = fP[((j * NR + rt) * NK2 + c2) * 64 + lane];
          bload(2 * c2, b[0]);
          bload(min(2 * c2 + 1, NK - 1), b[1]);
        };
        auto pchunks = [&](int c2, const float2 (&fp)[3][NR], const float (&b)[2][4]) {
          float f0[3][NR], f1[3][NR];
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int rt = 0; rt < NR; ++rt) {
              f0[j][rt] = fp[j][rt].x;
              f1[j][rt] = fp[j][rt].y;
            }
          vchunkb(b[0], f0);
          if (2 * c2 + 1 < NK) vchunkb(b[1], f1);
        };
        float2 pa[3][NR], pb[3][NR];
        float ba[2][4], bb[2][4];
        pload(0, pa, ba);
        for (int c2 = 0; c2 < NK2; c2 += 2) {
          __builtin_amdgcn_sched_barrier(0);
          pload(min(c2 + 1, NK2 - 1), pb, bb);
          __builtin_amdgcn_sched_barrier(0);
          pchunks(c2, pa, ba);
          __builtin_amdgcn_sched_barrier(0);
          pload(min(c2 + 2, NK2 - 1), pa, ba);
          __builtin_amdgcn_sched_barrier(0);
          if (c2 + 1 < NK2) pchunks(c2 + 1, pb, bb);
        }
        __builtin_amdgcn_sched_barrier(0);
      } else {
#pragma unroll VU
        for (int c = 0; c < NK; ++c) {
          vload(c, fa);
          vchunk(c, fa);
        }
      }
    } else {
      // lane (e, g) supplies B rows 16 c + 4 g .. + 3: node quad 4 c + g of each field
      auto bchunk = [&](int c, const uint4 (&fa)[3][NR]) {
        const int qd = 4 * c + g;
        const bool ok = 4 * c + 3 < NK || qd < NK;
        const int qr = ok ? qd : 0;
        float4 p4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(0, 4 * qr, e)]);
        float4 x4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(1, 4 * qr, e)]);
        float4 y4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(2, 4 * qr, e)]);
        float4 z4 = *reinterpret_cast<const float4 *>(&q_t[lqix<N>(3, 4 * qr, e)]);
        if (!ok) p4 = x4 = y4 = z4 = float4{0.f, 0.f, 0.f, 0.f};
        const float pv[4] = {p4.x, p4.y, p4.z, p4.w}, xv[4] = {x4.x, x4.y, x4.z, x4.w};
        const float yv[4] = {y4.x, y4.y, y4.z, y4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
        v4s urh, url, ush, usl, uth, utl, ph, pl;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          short h, l;
          split_bf16(rx * xv[v] + ry * yv[v] + rz * zv[v], h, l); urh[v] = h; url[v] = l;
          split_bf16(sx * xv[v] + sy * yv[v] + sz * zv[v], h, l); ush[v] = h; usl[v] = l;
          split_bf16(tx * xv[v] + ty * yv[v] + tz * zv[v], h, l); uth[v] = h; utl[v] = l;
          split_bf16(pv[v], h, l); ph[v] = h; pl[v] = l;
        }
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) {
          DGRTM_MF3(fa[0][rt], urh, url, cp[rt]);
          DGRTM_MF3(fa[1][rt], ush, usl, cp[rt]);
          DGRTM_MF3(fa[2][rt], uth, utl, cp[rt]);
          DGRTM_MF3(fa[0][rt], ph, pl, w0[rt]);
          DGRTM_MF3(fa[1][rt], ph, pl, w1[rt]);
          DGRTM_MF3(fa[2][rt], ph, pl, w2[rt]);
        }
      };
      auto bload = [&](int c, uint4 (&fa)[3][NR]) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int rt = 0; rt < NR; ++rt) fa[j][rt] = bD[((j * NR + rt) * DB::NK + c) * 64 + lane];
      };
      uint4 fa[3][NR];
      if constexpr (OPS_LDS != 1) {
        // fragments through the caches: two register buffers, as in the FP32 form
        uint4 fb[3][NR];
        bload(0, fa);
        for (int c = 0; c < DB::NK; c += 2) {
          __builtin_amdgcn_sched_barrier(0);
          bload(min(c + 1, DB::NK - 1), fb);
          __builtin_amdgcn_sched_barrier(0);
          bchunk(c, fa);
          __builtin_amdgcn_sched_barrier(0);
          bload(min(c + 2, DB::NK - 1), fa);
          __builtin_amdgcn_sched_barrier(0);
          if (c + 1 < DB::NK) bchunk(c + 1, fb);
        }
        __builtin_amdgcn_sched_barrier(0);
      } else {
#pragma unroll VU
        for (int c = 0; c < DB::NK; ++c) {
          bload(c, fa);
          bchunk(c, fa);
        }
      }
    }
    v4f rp[NR], rvx[NR], rvy[NR], rvz[NR];
    volume_to_rhs<NR>(gg, cp, w0, w1, w2, rp, rvx, rvy, rvz);

    if constexpr (OPS_LDS != 1) faces();

    // ---- surface: rp -= LIFT Pp (accumulated by the MFMA with -Pp), G_f = LIFT_f Pv, rv -= n_f G_f
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const FaceCtx &fc = fcs[f];
      nfx[f] = fc.nx; nfy[f] = fc.ny; nfz[f] = fc.nz;
      // boundary states without branches (cP = 1 rigid wall, -1 free surface, 0 otherwise; 0 on
      // every face when the boundary faces are replayed)
      const float cP = REPLAY ? 0.0f : (fc.nb == -1 ? 1.0f : (fc.nb == -3 ? -1.0f : 0.0f));
      const float(&tp)[TPN] = tpa[f];
      const float(&tv)[TPN] = tva[f];
      v4f G[NR];
#pragma unroll
      for (int rt = 0; rt < NR; ++rt) G[rt] = v4f{0.f, 0.f, 0.f, 0.f};
      if constexpr (PREC == 0) {
        // the face's penalties first, then its products (the fragment reads run ahead of the
        // products instead of waiting behind each chunk's penalty arithmetic)
        float mPp[FC], Pv[FC];
#pragma unroll
        for (int cc = 0; cc < FC; ++cc) {
          const bool sv = 4 * cc + 3 < Nfp || 4 * cc + g < Nfp;   // face node 4 cc + g exists
          const int node = sel4(g, T.fmask[f][4 * cc], T.fmask[f][min(4 * cc + 1, Nfp - 1)],
                                T.fmask[f][min(4 * cc + 2, Nfp - 1)], T.fmask[f][min(4 * cc + 3, Nfp - 1)]);
          const float pm = q_t[lqix<N>(0, node, e)];
          const float nvm = fc.nx * q_t[lqix<N>(1, node, e)] + fc.ny * q_t[lqix<N>(2, node, e)] +
                            fc.nz * q_t[lqix<N>(3, node, e)];
          const float pp = cP * pm + tp[cc];
          const float nvp = -(cP * nvm + tv[cc]);
          const float dp = pp - pm, dnv = nvp - nvm;
          mPp[cc] = sv ? -0.5f * rc2 * (dnv - fc.taup * dp) * fc.Fs : 0.0f;
          Pv[cc] = sv ? 0.5f * irho * (dp - fc.tauv * dnv) * fc.Fs : 0.0f;
        }
#pragma unroll
        for (int cc = 0; cc < FC; ++cc)
#pragma unroll
          for (int rt = 0; rt < NR; ++rt) {
            const float al = fL[(rt * 4 * FC + f * FC + cc) * 64 + lane];
            rp[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(al, mPp[cc], rp[rt], 0, 0, 0);
            G[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(al, Pv[cc], G[rt], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int cc = 0; cc < DB::FC; ++cc) {   // lane (e, g) takes face nodes 16 cc + 4 g + v
          v4s pph, ppl, pvh, pvl;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int s = 16 * cc + 4 * g + v;
            const bool sv = 16 * cc + 12 + v < Nfp || s < Nfp;
            const int node = sel4(g, T.fmask[f][min(16 * cc + v, Nfp - 1)], T.fmask[f][min(16 * cc + 4 + v, Nfp - 1)],
                                  T.fmask[f][min(16 * cc + 8 + v, Nfp - 1)], T.fmask[f][min(16 * cc + 12 + v, Nfp - 1)]);
            const float tps = tp[4 * cc + v], tvs = tv[4 * cc + v];
            const float pm = q_t[lqix<N>(0, node, e)];
            const float nvm = fc.nx * q_t[lqix<N>(1, node, e)] + fc.ny * q_t[lqix<N>(2, node, e)] +
                              fc.nz * q_t[lqix<N>(3, node, e)];
            const float pp = cP * pm + tps;
            const float nvp = -(cP * nvm + tvs);
            const float dp = pp - pm, dnv = nvp - nvm;
            const float mPp = sv ? -0.5f * rc2 * (dnv - fc.taup * dp) * fc.Fs : 0.0f;
            const float Pv = sv ? 0.5f * irho * (dp - fc.tauv * dnv) * fc.Fs : 0.0f;
            short h, l;
            split_bf16(mPp, h, l); pph[v] = h; ppl[v] = l;
            split_bf16(Pv, h, l); pvh[v] = h; pvl[v] = l;
          }
#pragma unroll
          for (int rt = 0; rt < NR; ++rt) {
            const uint4 al = bL[(rt * 4 * DB::FC + f * DB::FC + cc) * 64 + lane];
            DGRTM_MF3(al, pph, ppl, rp[rt]);
            DGRTM_MF3(al, pvh, pvl, G[rt]);
          }
        }
      }
#pragma unroll
      for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          rvx[rt][i] -= fc.nx * G[rt][i];
          rvy[rt][i] -= fc.ny * G[rt][i];
          rvz[rt][i] -= fc.nz * G[rt][i];
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    // the update prefetches the next row tile's rhs history where that costs no spills and pays
    // (measured: every step at N = 6, the forward and segment-record steps at N = 5)
    constexpr bool PF = BM == MODE_PLAIN || (N == 5 && BM == MODE_RECORD_SEG) || N >= 6;
    tile_tail<N, BM, true, false, false, false, BM != MODE_RHS_ONLY, PF>(a, sl, k, g, lev, sh, m, flag, q_t, e,
                                                                    gg[11], nfx, nfy, nfz, rp, rvx, rvy, rvz);
    // own-step traces of the new state (now in the state tile); the half-step ones went out per lane
    if constexpr (BM != MODE_RHS_ONLY) tile_traces<N, false>(a, sl, k, g, e, m, flag, q_t, nullptr, nfx, nfy, nfz);
    const int64_t nn = dyn ? 2 * nfirst + __builtin_amdgcn_readfirstlane(vnn) : nxt + nfirst;
    // every LDS read of this tile is done: the next tile's copies may land
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if (nxt < ntiles) {
      issue(nxt);
      if constexpr (OPS_LDS == 1) load_nb(nxt);
    }
    tile = nxt;
    nxt = nn;
  }
  if (dyn) {
    // the last work-group to finish clears the counters for the next launch (every wavefront of a
    // dyn launch gets here: its first tile is below W <= ntiles)
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t done = atomicAdd(ctr + 1, 1u);
      if (done + 1u == gridDim.x) {
        ctr[0] = 0u;
        ctr[1] = 0u;
      }
    }
  }
}

// Own-step traces of a whole field's state (at the start of a run or after a restore), as the step
// kernels write them: one wavefront per 16-element tile, lane (e, g) writes face g of element e as
// 16-byte stores of its p and n.v runs (the padding after the last face node gets zeros), reading
// the face nodes of the state per lane.
template <int N>
__global__ __launch_bounds__(256) void trace_init_kernel(const TraceInitArgs a) {
  constexpr Tab<N> T{};
  constexpr int Np = Tab<N>::Np, Nfp = Tab<N>::Nfp, NQ4 = node_quads(Np);
  constexpr int FS = Dims<N>::FS, TRC = Dims<N>::TRC, TRS = Dims<N>::TRS, TRF = Dims<N>::TRF;
  const int lane = threadIdx.x & 63;
  const int e = lane & 15, g = lane >> 4;
  const int64_t K = a.Ktot;
  const int64_t k = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + e;
  if (k >= K) return;
  if (!(a.eflag[k] & 1)) return;
  const int lev = level_of(a.lev_begin, a.L, k);
  const int64_t m = a.tau >> (a.L - lev);
  float gv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) gv[i] = a.geo[tix(kGeo, i, k)];
  // outward normal of face g (the step kernels' face contexts compute it the same way)
  float nx = g == 0 ? -gv[6] : (g == 1 ? -gv[3] : (g == 2 ? gv[0] + gv[3] + gv[6] : -gv[0]));
  float ny = g == 0 ? -gv[7] : (g == 1 ? -gv[4] : (g == 2 ? gv[1] + gv[4] + gv[7] : -gv[1]));
  float nz = g == 0 ? -gv[8] : (g == 1 ? -gv[5] : (g == 2 ? gv[2] + gv[5] + gv[8] : -gv[2]));
  const float Fs = sqrtf(nx * nx + ny * ny + nz * nz);
  const float inv = 1.0f / Fs;
  nx *= inv; ny *= inv; nz *= inv;
  float *tr = a.tr + (m & 1) * (int64_t)TRS * K + k * TRS + g * TRF;
#pragma unroll
  for (int j = 0; j < FS / 4; ++j) {
    float p[4], v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = 4 * j + u;
      p[u] = v[u] = 0.0f;
      if (s < Nfp) {
        const int node = sel4(g, T.fmask[0][s], T.fmask[1][s], T.fmask[2][s], T.fmask[3][s]);
        p[u] = a.q[qix(NQ4, 0, node, k)];
        v[u] = nx * a.q[qix(NQ4, 1, node, k)] + ny * a.q[qix(NQ4, 2, node, k)] + nz * a.q[qix(NQ4, 3, node, k)];
      }
    }
    *reinterpret_cast<float4 *>(tr + 4 * j) = float4{p[0], p[1], p[2], p[3]};
    *reinterpret_cast<float4 *>(tr + TRC + 4 * j) = float4{v[0], v[1], v[2], v[3]};
  }
}

template <int N>
__global__ __launch_bounds__(256) void seg_init_kernel(const SegInitArgs a) {
  constexpr int Np = Tab<N>::Np;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.Ktot) return;
  const int64_t K = a.Ktot;
  if (!(a.eflag[k] & 1)) return;
  const int lev = level_of(a.lev_begin, a.L, k);
  const int64_t kk = k - a.lev_begin[lev - 1];
  const int64_t Pl = level_end(a.lev_begin, a.L, lev) - a.lev_begin[lev - 1];
  const int64_t m0 = a.seg_m0[lev - 1];
  const float zs = a.condition ? a.geo[tix(kGeo, 11, k)] : 0.0f;
  const int64_t slab = (int64_t)state_row(Np) * K;
  for (int s = 1; s <= 2; ++s) {
    const int64_t ms = m0 - s;
    const float *R = a.ring + ((ms % 3 + 3) % 3) * slab;
    for (int n = 0; n < Np; ++n) {
      float v = 0.0f;
      if (ms >= 0 || a.history_before_start) {
        const float r0 = R[qix(node_quads(Np), 0, n, k)], r1 = R[qix(node_quads(Np), 1, n, k)];
        const float r2 = R[qix(node_quads(Np), 2, n, k)], r3 = R[qix(node_quads(Np), 3, n, k)];
        v = r0 - zs * (a.up[0] * r1 + a.up[1] * r2 + a.up[2] * r3);
      }
      a.seg_r[a.seg_r_off[lev - 1] + (2 - s) * Np * Pl + tix(Np, n, kk)] = v;
    }
  }
}

// one thread per 16-byte chunk of a boundary face's record row (FS / 4 chunks of p, then of -n.v)
template <int N>
__global__ __launch_bounds__(256) void bnd_record_kernel(const BndRecArgs a) {
  constexpr int FS = Dims<N>::FS, TRC = Dims<N>::TRC, TRS = Dims<N>::TRS, CH = FS / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_active * 2 * CH) return;
  const int64_t i = t / (2 * CH);
  const int comp = (int)(t % (2 * CH)) / CH, c = (int)(t % CH);
  const int sf = a.bface[i];
  const int64_t k = sf >> 2;
  const int f = sf & 3;
  const int lev = level_of(a.lev_begin, a.L, k);
  const int64_t j = (a.tau >> (a.L - lev)) + 1;   // own step reached by the launch at tau
  const float4 v = *reinterpret_cast<const float4 *>(a.tr + (j & 1) * (int64_t)TRS * a.Ktot + k * TRS +
                                                     f * Dims<N>::TRF + comp * TRC + 4 * c);
  const float sg = comp ? -1.0f : 1.0f;
  const int64_t b = i - a.bnd_begin[lev - 1];
  float *dst = a.rec + a.bnd_off[lev - 1] + (j * a.bnd_cnt[lev - 1] + b) * (2 * FS) + comp * FS + 4 * c;
  *reinterpret_cast<float4 *>(dst) = float4{sg * v.x, sg * v.y, sg * v.z, sg * v.w};
}

// the quadratic through r0, r1, r2 (the reversed-time rhs at t_f, t_f - dt_g, t_f - 2 dt_g),
// evaluated at t_f + dt_l and t_f + 2 dt_l (dt_l / dt_g = 2^(1 - l) for level l): ring slots 2, 1
__global__ __launch_bounds__(256) void replay_history_kernel(const float *r0, const float *r1, const float *r2,
                                                             float *ring, int64_t slab, int64_t tile_floats,
                                                             int L, ReplayLevels lb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= slab) return;
  const int lev = level_of(lb.lev_begin, L, (i / tile_floats) * 16);
  const double x0 = r0[i], x1 = r1[i], x2 = r2[i];
  const double rho = 1.0 / (double)(1LL << (lev - 1));
#pragma unroll
  for (int k = 1; k <= 2; ++k) {
    const double tau = k * rho;   // in units of dt_g after t_f
    const double l0 = 0.5 * (tau + 1.0) * (tau + 2.0), l1 = -tau * (tau + 2.0), l2 = 0.5 * tau * (tau + 1.0);
    ring[(k == 1 ? 2 : 1) * slab + i] = (float)(l0 * x0 + l1 * x1 + l2 * x2);
  }
}

__global__ void record_kernel(const float *q, int64_t K, const int64_t *pos, const float *l, int64_t n_rec, int Np,
                              float *out, int64_t stride) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rec) return;
  const int64_t k = pos[r];
  float acc = 0.0f;
  for (int n = 0; n < Np; ++n) acc += l[r * Np + n] * q[qix(node_quads(Np), 0, n, k)];
  out[r * stride] = acc;
}

__global__ void to_dev_kernel(int Np, int nf, const float *user, float *dev, const int64_t *s2u, int64_t K) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * Np) return;
  const int64_t k = t % K, n = t / K;
  const int64_t u = s2u[k];
  for (int c = 0; c < nf; ++c) dev[qix(node_quads(Np), c, n, k)] = u >= 0 ? user[(u * nf + c) * Np + n] : 0.0f;
}

__global__ void to_user_kernel(int Np, int nf, const float *dev, float *user, const int64_t *s2u, int64_t K) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * Np) return;
  const int64_t k = t % K, n = t / K;
  const int64_t u = s2u[k];
  if (u < 0) return;
  for (int c = 0; c < nf; ++c) user[(u * nf + c) * Np + n] = dev[qix(node_quads(Np), c, n, k)];
}

__global__ void img_user_kernel(int Np, const double *img, double *user, const int64_t *s2u, int64_t K, int acc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * Np) return;
  const int64_t k = t % K, n = t / K;
  const int64_t u = s2u[k];
  if (u < 0) return;
  const double v = img[tix(Np, n, k)];
  if (acc) user[u * Np + n] += v;
  else user[u * Np + n] = v;
}

__global__ void residual_kernel(const float *a, const float *b, int64_t n, double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)a[i] - (double)b[i];
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

__global__ void fill_f32_kernel(float *p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_f64_kernel(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

static int64_t device_cus() {
  static int64_t cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

template <int N, int MODE>
static hipError_t launch_step_mode(const StepArgs &a, hipStream_t st) {
  const int64_t groups = (a.k_end / 16 + 3) / 4;
  if constexpr (N >= 5) {
    // one work-group per CU: the operators (when they fit), the face-node map and one state tile
    // per wavefront
    constexpr size_t tiles = (size_t)4 * (DmaDims<N>::QW + DmaDims<N>::GW) * sizeof(float);
    constexpr size_t map = (size_t)4 * Dims<N>::TABW;
    constexpr size_t ops32 = (size_t)Dims<N>::OPS * sizeof(float);
    constexpr size_t opsb = (size_t)DimsB<N>::OPS_U4 * sizeof(uint4);
    // the lift fragments alone (when the volume fragments do not fit beside the tiles)
    constexpr size_t lift32 = ops32 - (size_t)3 * Dims<N>::NR * Dims<N>::NK * 64 * sizeof(float);
    constexpr size_t liftb = opsb - (size_t)3 * Dims<N>::NR * DimsB<N>::NK * 64 * sizeof(uint4);
    const dim3 grid1((unsigned)std::max<int64_t>(1, std::min(groups, a.max_groups > 0 ? a.max_groups : device_cus())),
                     (unsigned)a.nslots), block(256);
    auto go = [&](auto kern, size_t lds) -> hipError_t {
      hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, grid1, block, lds, st, a);
      return hipGetLastError();
    };
    if (a.precision == 1) {
      if constexpr (opsb + tiles + map <= 160 * 1024) return go(step_kernel_lowreg<N, MODE, 1, 1>, opsb + tiles);
      else if constexpr (liftb + tiles + map <= 160 * 1024) return go(step_kernel_lowreg<N, MODE, 2, 1>, liftb + tiles);
      else return go(step_kernel_lowreg<N, MODE, 0, 1>, tiles);
    }
    if constexpr (ops32 + tiles + map <= 160 * 1024) return go(step_kernel_lowreg<N, MODE, 1, 0>, ops32 + tiles);
    else if constexpr (lift32 + tiles + map <= 160 * 1024) return go(step_kernel_lowreg<N, MODE, 2, 0>, lift32 + tiles);
    else return go(step_kernel_lowreg<N, MODE, 0, 0>, tiles);
  } else {
    // one work-group per CU (its static LDS fills the CU); each loops over tiles.  A launch with
    // fewer than two tiles per wavefront of a full grid takes a smaller grid with two tiles per
    // wavefront (the second tile's copies overlap the first tile's work)
    const int64_t cus = a.max_groups > 0 ? a.max_groups : device_cus();
    const int64_t g2 = (a.k_end / 16 < 8 * cus) ? (a.k_end / 16 + 7) / 8 : groups;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min(g2, cus)), (unsigned)a.nslots), block(256);
    if (a.precision == 1)
      hipLaunchKernelGGL((step_kernel_dma<N, MODE, 1>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((step_kernel_dma<N, MODE, 0>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t launch_step_n(const StepArgs &a, hipStream_t st) {
  if (a.k_end <= 0 || a.nslots <= 0) return hipSuccess;
  if (a.nslots > kMaxSlots) return hipErrorInvalidValue;
  switch (a.mode) {
    case MODE_RHS_ONLY: return launch_step_mode<N, MODE_RHS_ONLY>(a, st);
    case MODE_IMAGE: return launch_step_mode<N, MODE_IMAGE>(a, st);
    case MODE_RECORD_SEG: return launch_step_mode<N, MODE_RECORD_SEG>(a, st);
    case MODE_PLAIN: return launch_step_mode<N, MODE_PLAIN>(a, st);
    case MODE_REPLAY_SEG: return launch_step_mode<N, MODE_REPLAY_SEG>(a, st);
    case MODE_RHS_REPLAY: return launch_step_mode<N, MODE_RHS_REPLAY>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// operator fragments in the MFMA A-operand lane order (see step_kernel_dma)
void build_op_fragments(int N, const float *Dr, const float *Ds, const float *Dt, const float *LIFT, float *out) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2, F = 4 * Nfp;
  const int NR = (Np + 15) / 16, NK = (Np + 3) / 4, FC = (Nfp + 3) / 4;
  const float *D[3] = {Dr, Ds, Dt};
  for (int j = 0; j < 3; ++j)
    for (int rt = 0; rt < NR; ++rt)
      for (int c = 0; c < NK; ++c)
        for (int l = 0; l < 64; ++l) {
          const int row = 16 * rt + (l & 15), col = 4 * c + (l >> 4);
          out[((j * NR + rt) * NK + c) * 64 + l] = (row < Np && col < Np) ? D[j][row * Np + col] : 0.0f;
        }
  float *L = out + 3 * NR * NK * 64;
  for (int rt = 0; rt < NR; ++rt)
    for (int f = 0; f < 4; ++f)
      for (int cc = 0; cc < FC; ++cc)
        for (int l = 0; l < 64; ++l) {
          const int row = 16 * rt + (l & 15), s = 4 * cc + (l >> 4);
          L[(rt * 4 * FC + f * FC + cc) * 64 + l] = (row < Np && s < Nfp) ? LIFT[row * F + f * Nfp + s] : 0.0f;
        }
  if (N >= 6) {
    // the volume fragments again, two column chunks per lane and 8-byte word: [3][NR][NK/2][64][2]
    // (read through the caches, one load per operator and row tile gives two chunks' A operands)
    const int NK2 = (NK + 1) / 2;
    float *P = L + NR * 4 * FC * 64;
    for (int j = 0; j < 3; ++j)
      for (int rt = 0; rt < NR; ++rt)
        for (int c2 = 0; c2 < NK2; ++c2)
          for (int l = 0; l < 64; ++l)
            for (int h = 0; h < 2; ++h) {
              const int c = 2 * c2 + h;
              const int row = 16 * rt + (l & 15), col = 4 * c + (l >> 4);
              P[(((j * NR + rt) * NK2 + c2) * 64 + l) * 2 + h] =
                  (c < NK && row < Np && col < Np) ? D[j][row * Np + col] : 0.0f;
            }
  }
}

static uint16_t host_bf16(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

static float host_bf16_value(uint16_t h) {
  const uint32_t b = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &b, 4);
  return x;
}

void build_op_fragments_bf16(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT,
                             uint32_t *out) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2, F = 4 * Nfp;
  const int NR = (Np + 15) / 16, NK = (Np + 15) / 16, FC = (Nfp + 15) / 16;
  auto put = [&](uint32_t *u, const double *vals) {  // 4 values -> hi pair, lo pair
    uint16_t h[4], l[4];
    for (int v = 0; v < 4; ++v) {
      h[v] = host_bf16((float)vals[v]);
      l[v] = host_bf16((float)(vals[v] - (double)host_bf16_value(h[v])));
    }
    u[0] = h[0] | ((uint32_t)h[1] << 16);
    u[1] = h[2] | ((uint32_t)h[3] << 16);
    u[2] = l[0] | ((uint32_t)l[1] << 16);
    u[3] = l[2] | ((uint32_t)l[3] << 16);
  };
  const double *D[3] = {Dr, Ds, Dt};
  for (int j = 0; j < 3; ++j)
    for (int rt = 0; rt < NR; ++rt)
      for (int c = 0; c < NK; ++c)
        for (int l = 0; l < 64; ++l) {
          const int row = 16 * rt + (l & 15);
          double vals[4];
          for (int v = 0; v < 4; ++v) {
            const int col = 16 * c + 4 * (l >> 4) + v;
            vals[v] = (row < Np && col < Np) ? D[j][row * Np + col] : 0.0;
          }
          put(out + 4 * (((j * NR + rt) * NK + c) * 64 + l), vals);
        }
  uint32_t *L = out + 4 * (3 * NR * NK * 64);
  for (int rt = 0; rt < NR; ++rt)
    for (int f = 0; f < 4; ++f)
      for (int cc = 0; cc < FC; ++cc)
        for (int l = 0; l < 64; ++l) {
          const int row = 16 * rt + (l & 15);
          double vals[4];
          for (int v = 0; v < 4; ++v) {
            const int s = 16 * cc + 4 * (l >> 4) + v;
            vals[v] = (row < Np && s < Nfp) ? LIFT[row * F + f * Nfp + s] : 0.0;
          }
          put(L + 4 * ((rt * 4 * FC + f * FC + cc) * 64 + l), vals);
        }
}

int64_t op_fragment_bf16_words(int N) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  const int NR = (Np + 15) / 16, NK = (Np + 15) / 16, FC = (Nfp + 15) / 16;
  return (int64_t)(3 * NR * NK + NR * 4 * FC) * 64 * 4;
}

int64_t op_fragment_floats(int N) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  const int NR = (Np + 15) / 16, NK = (Np + 3) / 4, FC = (Nfp + 3) / 4;
  const int64_t paired = N >= 6 ? (int64_t)3 * NR * ((NK + 1) / 2) * 64 * 2 : 0;
  return (int64_t)(3 * NR * NK + NR * 4 * FC) * 64 + paired;
}

hipError_t launch_step(int N, const StepArgs &a, hipStream_t st) {
  switch (N) {
    case 1: return launch_step_n<1>(a, st);
    case 2: return launch_step_n<2>(a, st);
    case 3: return launch_step_n<3>(a, st);
    case 4: return launch_step_n<4>(a, st);
    case 5: return launch_step_n<5>(a, st);
    case 6: return launch_step_n<6>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_trace_init(int N, const TraceInitArgs &a, hipStream_t st) {
  const dim3 grid(blocks_for(a.Ktot, 64)), block(256);   // four 16-element tiles per work-group
  switch (N) {
    case 1: hipLaunchKernelGGL(trace_init_kernel<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(trace_init_kernel<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(trace_init_kernel<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(trace_init_kernel<4>, grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL(trace_init_kernel<5>, grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL(trace_init_kernel<6>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_seg_init(int N, const SegInitArgs &a, hipStream_t st) {
  const dim3 grid(blocks_for(a.Ktot, 256)), block(256);
  switch (N) {
    case 1: hipLaunchKernelGGL(seg_init_kernel<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(seg_init_kernel<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(seg_init_kernel<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(seg_init_kernel<4>, grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL(seg_init_kernel<5>, grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL(seg_init_kernel<6>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_record(int N, const float *q, int64_t Ktot, const int64_t *rec_pos, const float *rec_l, int64_t n_rec,
                         float *out, int64_t out_stride, hipStream_t st) {
  if (n_rec <= 0) return hipSuccess;
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  hipLaunchKernelGGL(record_kernel, dim3(blocks_for(n_rec, 256)), dim3(256), 0, st, q, Ktot, rec_pos, rec_l, n_rec, Np,
                     out, out_stride);
  return hipGetLastError();
}

hipError_t launch_to_device_layout(int Np, int nf, const float *user, float *dev, const int64_t *s2u, int64_t K,
                                   hipStream_t st) {
  if (nf != 4) return hipErrorInvalidValue;   // the quad layout holds the four fields
  hipLaunchKernelGGL(to_dev_kernel, dim3(blocks_for(K * Np, 256)), dim3(256), 0, st, Np, nf, user, dev, s2u, K);
  return hipGetLastError();
}
hipError_t launch_to_user_layout(int Np, int nf, const float *dev, float *user, const int64_t *s2u, int64_t K,
                                 hipStream_t st) {
  if (nf != 4) return hipErrorInvalidValue;   // the quad layout holds the four fields
  hipLaunchKernelGGL(to_user_kernel, dim3(blocks_for(K * Np, 256)), dim3(256), 0, st, Np, nf, dev, user, s2u, K);
  return hipGetLastError();
}
hipError_t launch_image_to_user(int Np, const double *img, double *user, const int64_t *s2u, int64_t K, int acc,
                                hipStream_t st) {
  hipLaunchKernelGGL(img_user_kernel, dim3(blocks_for(K * Np, 256)), dim3(256), 0, st, Np, img, user, s2u, K, acc);
  return hipGetLastError();
}
hipError_t launch_residual(const float *a, const float *b, int64_t n, double *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  unsigned nb = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(256), 0, st, a, b, n, out);
  return hipGetLastError();
}
hipError_t launch_bnd_record(int N, const BndRecArgs &a, hipStream_t st) {
  if (a.n_active <= 0) return hipSuccess;
  auto go = [&](auto kern, int FS) {
    hipLaunchKernelGGL(kern, dim3(blocks_for(a.n_active * 2 * (FS / 4), 256)), dim3(256), 0, st, a);
  };
  switch (N) {
    case 1: go(bnd_record_kernel<1>, Dims<1>::FS); break;
    case 2: go(bnd_record_kernel<2>, Dims<2>::FS); break;
    case 3: go(bnd_record_kernel<3>, Dims<3>::FS); break;
    case 4: go(bnd_record_kernel<4>, Dims<4>::FS); break;
    case 5: go(bnd_record_kernel<5>, Dims<5>::FS); break;
    case 6: go(bnd_record_kernel<6>, Dims<6>::FS); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_replay_history(int Np, const float *r0, const float *r1, const float *r2, float *ring, int64_t Ktot,
                                 int L, const int64_t *lev_begin, hipStream_t st) {
  const int64_t slab = (int64_t)state_row(Np) * Ktot;
  if (slab <= 0) return hipSuccess;
  ReplayLevels lb;
  for (int i = 0; i <= kMaxLevels; ++i) lb.lev_begin[i] = lev_begin[i];
  hipLaunchKernelGGL(replay_history_kernel, dim3(blocks_for(slab, 256)), dim3(256), 0, st, r0, r1, r2, ring, slab,
                     (int64_t)16 * state_row(Np), L, lb);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace dgrtm
