// Split-FP16 MFMA product of the eigenbasis mixers (Golden et al., JuliQAOA, SC-W 2023,
// Sec. 2.1: e^{-i beta H_M} = V e^{-i beta D} V^{-1}; Sec. 2.2: the products with V and V^{-1}
// dominate the cost of the mixers without a product form).
//
// One product C = op(V) Psi for every angle set at once: Psi is the N x cols real matrix of
// the states (real and imaginary parts as separate columns), op(V) is V^T (into the
// eigenbasis) or V (back). FP32 accumulation of FP16 matrix-core products: every operand is
// split as x = x_h + 2^-11 x_l with x_h = fp16(x), x_l = fp16(2^11 (x - x_h)) (the scaled low
// half stays clear of FP16 subnormals), and
//     C = V_h Psi_h + 2^-11 (V_h Psi_l + V_l Psi_h)          (+ 2^-22 V_l Psi_l, dropped)
// with the hi x hi products and the cross products in two FP32 accumulators, three MFMAs per
// block. The dropped term is 2^-22 relative.
//
// Tiling (gfx950, v_mfma_f32_32x32x16_f16): a workgroup of 256 threads (one wave per SIMD)
// owns a tile of 128 state columns x 256 rows of C; wave w computes all 128 columns (4 blocks of
// 32) for its own 64 rows (2 blocks of 32). The MFMA's first operand is the state (K-contiguous
// per column), the second the matrix (K-contiguous per row of op(V)), so the accumulator of a
// lane holds 4 consecutive state columns per group for one row of C: the real and imaginary
// columns of an angle set sit in the same lane, and stores of C run over consecutive rows.
//
// Operand paths. The matrix is constant, so it is kept in the fragment-major layout
// (split_frag_offset): a wave's fragment of one row block and K step is one contiguous 1 KB
// global load straight into registers, prefetched seven K steps ahead; rows are private to a
// wave, so nothing of the matrix passes through LDS. The state is shared by the four waves: its
// K tiles of 32 (the blocked layout, one contiguous 8 KB block per plane) are copied through
// registers into one of two LDS stages while the other stage is multiplied out; its fragments
// are read from LDS (chunk-swizzled rows: conflict-free 16-byte reads). Per K step of 16 a wave
// issues 24 MFMAs (4 x 2 blocks, three products each) against 4 KB of matrix loads and 8 KB of
// LDS reads.
//
// Operands are zero-padded so every access is in bounds and unguarded: the matrix planes hold
// Mp = roundup(M, 256) rows of Kp = roundup(K, 128) halves, the state planes Ncp =
// roundup(cols, 128) columns of Kp halves. The tile configuration is fixed at build time, so
// results do not depend on the process or the run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qaoa_internal.h"

namespace qaoa {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int GN = SPLIT_TILE;           // state columns per workgroup
constexpr int GM = SPLIT_MTILE;          // rows of C per workgroup
constexpr int GK = SPLIT_KTILE;          // K tile of one LDS stage
constexpr int BLK = GN * GK;             // halves per state block (one plane, one column tile, one K tile)
constexpr int STAGE = 2 * BLK;           // halves per LDS stage (hi and lo planes)
constexpr int NB = 4, MB = 2;            // 32-blocks per wave: state columns, rows of C
constexpr int DV = 7;                    // matrix prefetch depth in K steps (a ring of 8 slots)

// Chunk swizzle of a block: row r holds its four 16-byte chunks in the order c ^ ((r >> 2) & 3),
// so the 16-byte fragment reads of 16 consecutive rows hit 64 distinct banks.
__device__ __forceinline__ int swz(int r, int c) { return c ^ ((r >> 2) & 3); }

__device__ __forceinline__ h8 sfrag(const _Float16 *buf, int plane, int r, int k) {
  return *(const h8 *)(buf + plane * BLK + r * GK + 8 * swz(r, k >> 3));
}

// One wave's matrix fragments of one K step: rows blocks 0 and 1 of the wave, hi and lo.
struct VFr {
  h8 h[MB], l[MB];
};

}  // namespace

// The hi x hi products (acc) and the two cross products (cx, each summed at its own scale) of
// this workgroup's tile (per lane: NB x MB blocks of 16 floats); op(V) Psi = acc + 2^-11 cx,
// joined by the caller's epilogue one element at a time (the accumulators stay in the matrix
// registers until then).
__device__ __forceinline__ void split_gemm_tile(const _Float16 *__restrict__ st_h, const _Float16 *__restrict__ st_l,
                                                const _Float16 *__restrict__ m_h, const _Float16 *__restrict__ m_l,
                                                int64_t kp, int ct, int rt, int kt0, int kt1, _Float16 *lds,
                                                f16v (&acc)[NB][MB], f16v (&cx)[NB][MB]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nk = (int)(kp / GK), nks = 2 * nk;
  const int klast = kt1 - 1, slast = 2 * kt1 - 1;  // last K tile and K step of the range
  // state: block (ct, kt) of each plane is 8 KB contiguous; wave w copies its 2 KB of each
  // through two sets of four registers (a tile is loaded two tiles before it is stored)
  const uint4 *sh = (const uint4 *)(st_h + (int64_t)ct * nk * BLK) + w * 128 + lane;
  const uint4 *sl = (const uint4 *)(st_l + (int64_t)ct * nk * BLK) + w * 128 + lane;
  uint4 sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3;
#define SLOAD(kt, r0, r1, r2, r3)                        \
  do {                                                   \
    const int64_t o_ = (int64_t)(kt) * (BLK / 8);        \
    r0 = sh[o_];                                         \
    r1 = sh[o_ + 64];                                    \
    r2 = sl[o_];                                         \
    r3 = sl[o_ + 64];                                    \
  } while (0)
#define SSTORE(stage, r0, r1, r2, r3)                                      \
  do {                                                                     \
    uint4 *d_ = (uint4 *)(lds + (stage) * STAGE) + w * 128 + lane;         \
    d_[0] = r0;                                                            \
    d_[64] = r1;                                                           \
    d_[BLK / 8] = r2;                                                      \
    d_[BLK / 8 + 64] = r3;                                                 \
  } while (0)
  // matrix: row blocks 8 rt + 2 w and + 1; chunk (rb, ks) at ((rb * nks + ks) * 64 + lane) * 8 halves
  const int rb0 = rt * (GM / 32) + MB * w;
  const h8 *vh = (const h8 *)m_h + (int64_t)rb0 * nks * 64 + lane;
  const h8 *vl = (const h8 *)m_l + (int64_t)rb0 * nks * 64 + lane;
  const int64_t vrow = (int64_t)nks * 64;  // h8 elements between consecutive row blocks
  auto vload = [&](VFr &f, int ks) {
#pragma unroll
    for (int j = 0; j < MB; j++) {
      f.h[j] = vh[j * vrow + ks * 64];
      f.l[j] = vl[j * vrow + ks * 64];
    }
  };
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int j = 0; j < MB; j++) {
      acc[i][j] = f16v{};
      cx[i][j] = f16v{};
    }
  const int fr = lane & 31, fk = 8 * (lane >> 5);
  // state fragments of one K step (hi and lo of the 4 column blocks), double-buffered: the next
  // step's are read from LDS while this step's MFMAs run
  struct SFr {
    h8 h[NB], l[NB];
  };
  auto sread = [&](SFr &f, const _Float16 *buf, int koff) {
#pragma unroll
    for (int i = 0; i < NB; i++) {
      f.h[i] = sfrag(buf, 0, 32 * i + fr, koff + fk);
      f.l[i] = sfrag(buf, 1, 32 * i + fr, koff + fk);
    }
  };
  auto mfmas = [&](const SFr &a, const VFr &b) {
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < MB; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.h[i], b.h[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < MB; j++) cx[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.l[i], b.h[j], cx[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
      for (int j = 0; j < MB; j++) cx[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.h[i], b.l[j], cx[i][j], 0, 0, 0);
  };
  // K tiles [kt0, kt1) (multiples of 4, at least 4 tiles). Prologue: tiles kt0 and kt0 + 1 into LDS stages 0 and 1, kt0 + 2 and kt0 + 3 into
  // the register sets, the matrix fragments of the first DV steps (past-the-end tile and step
  // indices are clamped: they re-read the range's last one, never used)
  VFr ring[DV + 1];
#pragma unroll
  for (int d = 0; d < DV; d++) vload(ring[d], 2 * kt0 + d);
  SLOAD(kt0, sa0, sa1, sa2, sa3);
  SLOAD(kt0 + 1, sb0, sb1, sb2, sb3);
  SSTORE(0, sa0, sa1, sa2, sa3);
  SSTORE(1, sb0, sb1, sb2, sb3);
  SLOAD(kt0 + 2, sa0, sa1, sa2, sa3);
  SLOAD(kt0 + 3, sb0, sb1, sb2, sb3);
  __syncthreads();
  SFr f0, f1;
  sread(f0, lds, 0);
  // Three LDS stages, K tiles in fours (the range is a multiple of 4) so that register sets and matrix
  // slots are constants. Tile k2 (stage k2 % 3): one barrier (stages k2 and k2 + 1 written by
  // every wave, stage k2 + 2 = k2 - 1 free); tile k2 + 2 goes from its registers to LDS and
  // tile k2 + 4 is loaded into them; step 2 k2 multiplies fragments read during the previous
  // step while it reads those of step 2 k2 + 1, which in turn reads tile k2 + 1's first ones.
  // The matrix fragments of step s are loaded DV steps ahead into the slot step s - 1 used.
  for (int kt = kt0; kt < kt1; kt += 4) {
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int k2 = kt + u, kr = k2 - kt0;  // kr: position in the range (stage index)
      __syncthreads();
      if ((u & 1) == 0) {
        SSTORE((kr + 2) % 3, sa0, sa1, sa2, sa3);
        SLOAD(min(k2 + 4, klast), sa0, sa1, sa2, sa3);
      } else {
        SSTORE((kr + 2) % 3, sb0, sb1, sb2, sb3);
        SLOAD(min(k2 + 4, klast), sb0, sb1, sb2, sb3);
      }
      const _Float16 *cur = lds + (kr % 3) * STAGE, *nxt = lds + ((kr + 1) % 3) * STAGE;
      const int s0 = 2 * k2;
      sread(f1, cur, 16);
      vload(ring[(2 * u + DV) & 7], min(s0 + DV, slast));
      mfmas(f0, ring[2 * u]);
      sread(f0, nxt, 0);
      vload(ring[(2 * u + 1 + DV) & 7], min(s0 + 1 + DV, slast));
      mfmas(f1, ring[2 * u + 1]);
      // Issue order of this tile (the region between two barriers): the LDS stores first, then
      // the 48 MFMAs with the 8 + 8 fragment reads and the 12 global loads slotted between
      // them one at a time, so every load is issued early and its latency hides behind the
      // matrix instructions (left alone, the scheduler sinks the loads to the end of the
      // region to shorten register lifetimes, and the next tile waits on them).
      __builtin_amdgcn_sched_group_barrier(0x200, 4, 0);  // DS write: tile k2 + 2 to LDS
#pragma unroll
      for (int g = 0; g < 8; g++) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read: step 2 k2 + 1 fragments
      }
#pragma unroll
      for (int g = 0; g < 12; g++) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read: state tile, matrix slots
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
#pragma unroll
      for (int g = 0; g < 8; g++) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read: tile k2 + 1 fragments
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
    }
  }
#undef SLOAD
#undef SSTORE
  __syncthreads();  // every wave is done with the stages before the epilogue reuses LDS
}

template <typename TT>
__device__ __forceinline__ uint32_t tab_at(const void *t, int64_t x) {
  return (uint32_t)((const TT *)t)[x];
}

// Sine and cosine of x (FP64 angle of modest size, |x| < 2^20): x = q pi/2 + r with |r| <= pi/4
// in FP64 (pi/2 as a two-part constant), then the Taylor polynomials of sin and cos in FP32 on r
// (through r^9 and r^10: truncation below 2e-9 on |r| <= pi/4) and the quadrant q mod 4. No
// table and no large-argument path, so nothing leaves the registers.
__device__ __forceinline__ void sincos_reduced(double x, float &sn, float &cs) {
  const double q = rint(x * 0.6366197723675814);
  const float r = (float)fma(-q, 6.123233995736766e-17, fma(-q, 1.5707963267948966, x));
  const float r2 = r * r;
  float s = fmaf(r2, 2.7557319e-6f, -1.9841270e-4f);
  s = fmaf(r2, s, 8.3333333e-3f);
  s = fmaf(r2, s, -1.6666667e-1f);
  s = fmaf(r2 * r, s, r);
  float c = fmaf(r2, -2.7557319e-7f, 2.4801587e-5f);
  c = fmaf(r2, c, -1.3888889e-3f);
  c = fmaf(r2, c, 4.1666667e-2f);
  c = fmaf(r2, c, -0.5f);
  c = fmaf(r2, c, 1.0f);
  const int k = (int)q & 3;
  sn = k == 0 ? s : (k == 1 ? c : (k == 2 ? -s : -c));
  cs = k == 0 ? c : (k == 1 ? -s : (k == 2 ? -c : s));
}

// Sum v over the 32 rows of this lane's half-wave (lanes with the same lane >> 5), in a fixed
// butterfly order; every lane of the half ends with the sum.
__device__ __forceinline__ double rows_sum(double v) {
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// Epilogue of one workgroup tile (rows r * GM.., columns c * GN..) of product op(V) Psi =
// acc + 2^-11 cx (per lane, NB x MB blocks of 16 floats): the elementwise step of MODE on each
// element, its FP32 or next-product output, and the tile's FP64 row sums per angle set. LDS
// (gsm) must be free. Column blocks [IB, IE) only (each block's angle sets are complete in it).
template <int MODE, typename TT, int IB = 0, int IE = NB>
__device__ __forceinline__ void split_epilogue(f16v (&acc)[NB][MB], f16v (&cx)[NB][MB], int r, int c, int M, int cols,
                                               const SplitEpi &e, unsigned char *gsm) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = r * GM + w * (32 * MB), n0 = c * GN;
  constexpr bool RED = MODE == SE_LAST || MODE == SE_REIG || MODE == SE_RPHASE;
  constexpr int SW = GN / 2;     // angle sets of the tile
  double *sred = (double *)gsm;  // [wave][SW sets][2]: per-wave row sums, reduced in wave order
  // per-row data of the wave's two row blocks
  double dd[MB], cvv[MB];
  uint32_t cii[MB];
#pragma unroll
  for (int jj = 0; jj < MB; jj++) {
    const int m = m0 + 32 * jj + (lane & 31);
    dd[jj] = cvv[jj] = 0.0;
    cii[jj] = 0;
    if (m >= M) continue;
    if constexpr (MODE == SE_EIG || MODE == SE_REIG) dd[jj] = e.D[m];
    if constexpr (MODE == SE_PHASE || MODE == SE_LAST || MODE == SE_RPHASE) {
      cii[jj] = tab_at<TT>(e.table, m);
      cvv[jj] = e.vals[cii[jj]];
    }
  }
  const float inv = 1.0f / 2048.0f;
  // one column block (16 angle sets) at a time: its sums over the wave's rows are complete
  // after both row blocks, so only 8 (or 16) FP64 sums are live
#pragma unroll
  for (int i = IB; i < IE; i++) {
    double red0[4][2], red1[4][2];
#pragma unroll
    for (int g = 0; g < 4; g++)
#pragma unroll
      for (int h = 0; h < 2; h++) red0[g][h] = red1[g][h] = 0.0;
#pragma unroll
    for (int jj = 0; jj < MB; jj++) {
      const int m = m0 + 32 * jj + (lane & 31);
      if (m >= M) continue;
      const double d = dd[jj], cv = cvv[jj];
      const uint32_t ci = cii[jj];
#pragma unroll
      for (int g = 0; g < 4; g++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int n = n0 + 32 * i + 8 * g + 4 * (lane >> 5) + 2 * h;  // real-part column, even
          if (n >= cols) continue;
          const int sidx = n >> 1;
          float re = fmaf(cx[i][jj][4 * g + 2 * h], inv, acc[i][jj][4 * g + 2 * h]);
          float im = fmaf(cx[i][jj][4 * g + 2 * h + 1], inv, acc[i][jj][4 * g + 2 * h + 1]);
          if constexpr (MODE == SE_PLAIN) {
            e.C[m + (int64_t)n * e.ldc] = re;
            e.C[m + (int64_t)(n + 1) * e.ldc] = im;
            continue;
          }
          if constexpr (MODE == SE_REIG) {
            const float ta = e.ckr[m + (int64_t)n * e.ldc], tb = e.ckr[m + (int64_t)(n + 1) * e.ldc];
            red0[g][h] += d * ((double)re * tb - (double)im * ta);
          }
          if constexpr (MODE == SE_RPHASE) {
            const float pa = e.ckr[m + (int64_t)n * e.ldc], pb = e.ckr[m + (int64_t)(n + 1) * e.ldc];
            red0[g][h] += (cv - e.c0) * ((double)re * pb - (double)im * pa);
          }
          if constexpr (MODE == SE_LAST) {
            const double pr = (double)re * re + (double)im * im;
            red0[g][h] += pr * cv;
            red1[g][h] += pr;
            e.C[m + (int64_t)n * e.ldc] = re;
            e.C[m + (int64_t)(n + 1) * e.ldc] = im;
            if (e.bout) {
              const float k = (float)(cv - e.c0);
              split_emit(e.bout, e.bld, e.bplane, m, sidx, k * re, k * im);
            }
            continue;
          }
          if constexpr (MODE == SE_EIG || MODE == SE_REIG) {
            // e^{-+i beta_s d} (angle in FP64; the result is rounded to FP32 anyway)
            float sn, cs;
            sincos_reduced((MODE == SE_EIG ? -1.0 : 1.0) * e.betas[sidx] * d, sn, cs);
            const float a = re, bb = im;
            re = a * cs - bb * sn;
            im = a * sn + bb * cs;
          }
          if constexpr (MODE == SE_PHASE || MODE == SE_RPHASE) {
            if (MODE == SE_RPHASE && !e.bout) continue;
            const float2 l = e.luts[(int64_t)sidx * e.lut_len + ci];
            const float a = re, bb = im;
            re = a * l.x - bb * l.y;
            im = a * l.y + bb * l.x;
          }
          if constexpr (MODE == SE_EIG || MODE == SE_PHASE) {
            if (e.ck) {
              e.ck[m + (int64_t)n * e.ldc] = re;
              e.ck[m + (int64_t)(n + 1) * e.ldc] = im;
            }
          }
          split_emit(e.bout, e.bld, e.bplane, m, sidx, re, im);
        }
    }
    if constexpr (RED) {
      // rows of this wave -> lanes 0 and 32
#pragma unroll
      for (int g = 0; g < 4; g++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const double s0 = rows_sum(red0[g][h]);
          const double s1 = MODE == SE_LAST ? rows_sum(red1[g][h]) : 0.0;
          if ((lane & 31) == 0) {
            const int sl = (32 * i + 8 * g + 4 * (lane >> 5) + 2 * h) >> 1;  // set within the tile's columns
            sred[(w * SW + sl) * 2] = s0;
            sred[(w * SW + sl) * 2 + 1] = s1;
          }
        }
    }
    // the scheduler may not hoist the next block's loads and transcendentals above this one
    // (that would keep them all live at once)
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (RED) {
    __syncthreads();
    if (t >= 16 * IB && t < 16 * IE) {
      const int s = c * SW + t;
      if (2 * s < cols) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int ww = 0; ww < 4; ww++) {
          a0 += sred[(ww * SW + t) * 2];
          a1 += sred[(ww * SW + t) * 2 + 1];
        }
        e.part0[(int64_t)s * e.nblk + r] = a0;
        if (MODE == SE_LAST) e.part1[(int64_t)s * e.nblk + r] = a1;
      }
    }
  }
}

// The product of one workgroup tile with epilogue MODE. Workgroup b runs on XCD b % 8
// (round-robin dispatch); each XCD takes the row tiles r = x (mod 8) and, for each, every
// column tile in consecutive workgroups, so the workgroups resident on one XCD at a time share
// each matrix row tile (8 column tiles) and each state column tile (4 row tiles) through that
// XCD's L2.
template <int MODE, typename TT>
__global__ __launch_bounds__(256, 1) void k_split_gemm(const _Float16 *__restrict__ st_h,
                                                       const _Float16 *__restrict__ st_l,
                                                       const _Float16 *__restrict__ m_h,
                                                       const _Float16 *__restrict__ m_l, int64_t kp, int M,
                                                       int cols, const SplitEpi e) {
  extern __shared__ __align__(16) unsigned char gsm[];
  _Float16 *lds = (_Float16 *)gsm;
  const int ctiles = (cols + GN - 1) / GN, mtiles = (M + GM - 1) / GM;
  const int b = blockIdx.x, x = b & 7, j = b >> 3;
  const int r = 8 * (j / ctiles) + x, c = j % ctiles;
  if (r >= mtiles) return;
  f16v acc[NB][MB], cx[NB][MB];
  split_gemm_tile(st_h, st_l, m_h, m_l, kp, c, r, 0, (int)(kp / GK), lds, acc, cx);
  split_epilogue<MODE, TT>(acc, cx, r, c, M, cols, e, gsm);
}

// ---- XCD-balanced schedule
//
// With one 256-row x 128-column tile per CU at a time, a product of more tiles than CUs runs in
// rounds, and the last round is partly empty (M = 12870 rows, 1024 columns: 51 x 8 tiles on 256
// CUs take two full rounds for 1.59 rounds of work). The balanced schedule keeps 32 workgroups
// per XCD at a time and splits the work evenly over the XCDs along K: a super-tile is RPS =
// 32 / ctiles row tiles times every column tile, processed by the 32 workgroups of one XCD in
// step (so each matrix row tile is shared by the column tiles and each state tile by the row
// tiles through that XCD's L2, as in the plain schedule); the S super-tiles x NQ K quads (4 K
// tiles each) are cut into 8 equal ranges, one per XCD. A super-tile cut by a range boundary is computed in two K
// pieces on two XCDs; each piece stores its partial sums to the workspace, and a second
// kernel adds the two (head piece first) and runs the epilogue. The cuts depend only on the
// product's shape, so results do not depend on the process or the run.
struct BalShape {
  int mtiles, ctiles, rps, S, nq;
};

__host__ __device__ inline bool bal_shape(int M, int cols, int64_t kp, BalShape &b) {
  b.mtiles = (M + GM - 1) / GM;
  b.ctiles = (cols + GN - 1) / GN;
  b.nq = (int)(kp / (4 * GK));
  if (b.ctiles > 32) return false;
  b.rps = 32 / b.ctiles;
  b.S = (b.mtiles + b.rps - 1) / b.rps;
  return b.S > 8 && b.S % 8 != 0;
}

// First K quad (global index super-tile * nq + quad) of XCD x's range; x = 0..8.
__host__ __device__ inline int64_t bal_cut(const BalShape &b, int x) { return (int64_t)x * b.S * b.nq / 8; }

constexpr int BAL_SLOT = NB * MB * 16 * 256;  // floats of one tile's partial sums

// Partial-sum slot of the piece of cut xb (1..7) that ends at the cut (part 0) or starts there
// (part 1), for workgroup j of its XCD.
__device__ __forceinline__ float *bal_slot(float *ws, int xb, int part, int j) {
  return ws + ((int64_t)((xb - 1) * 2 + part) * 32 + j) * BAL_SLOT;
}

// Pieces an XCD's range can touch: at most ceil(S / 8) + 1 super-tiles.
__host__ __device__ inline int bal_pmax(const BalShape &b) { return (b.S + 7) / 8 + 1; }

// Workgroup b: XCD x = b % 8 (round-robin dispatch), piece pi = (b / 8) / 32 of that XCD's
// range, tile j = (b / 8) % 32 of the super-tile. The workgroups of piece pi + 1 are queued
// behind those of piece pi on the XCD, so its 32 CUs move from piece to piece together.
template <int MODE, typename TT>
__global__ __launch_bounds__(256, 1) void k_split_gemm_bal(const _Float16 *__restrict__ st_h,
                                                           const _Float16 *__restrict__ st_l,
                                                           const _Float16 *__restrict__ m_h,
                                                           const _Float16 *__restrict__ m_l, int64_t kp, int M,
                                                           int cols, const SplitEpi e) {
  extern __shared__ __align__(16) unsigned char gsm[];
  _Float16 *lds = (_Float16 *)gsm;
  BalShape bs;
  (void)bal_shape(M, cols, kp, bs);
  const int b = blockIdx.x, x = b & 7, pi = (b >> 3) >> 5, j = (b >> 3) & 31;
  const int rho = j / bs.ctiles, c = j % bs.ctiles;
  if (rho >= bs.rps) return;
  const int64_t g0 = bal_cut(bs, x), g1 = bal_cut(bs, x + 1);
  const int64_t gs = pi == 0 ? g0 : (g0 / bs.nq + pi) * bs.nq;
  if (gs >= g1) return;
  const int64_t ge = (gs / bs.nq + 1) * bs.nq < g1 ? (gs / bs.nq + 1) * bs.nq : g1;
  const int q0 = (int)(gs % bs.nq), q1 = q0 + (int)(ge - gs);
  const int r = (int)(gs / bs.nq) * bs.rps + rho;
  if (r >= bs.mtiles) return;
  f16v acc[NB][MB], cx[NB][MB];
  split_gemm_tile(st_h, st_l, m_h, m_l, kp, c, r, 4 * q0, 4 * q1, lds, acc, cx);
  if (q0 == 0 && q1 == bs.nq) {
    split_epilogue<MODE, TT>(acc, cx, r, c, M, cols, e, gsm);
    return;
  }
  // a piece of a cut super-tile: its partial sums, element-major (coalesced per element)
  const int t = threadIdx.x;
  const float inv = 1.0f / 2048.0f;
  float *slot = q0 == 0 ? bal_slot(e.ws, x + 1, 0, j) : bal_slot(e.ws, x, 1, j);
#pragma unroll
  for (int i = 0; i < NB; i++)
#pragma unroll
    for (int jj = 0; jj < MB; jj++)
#pragma unroll
      for (int v = 0; v < 16; v++)
        slot[(int64_t)((i * MB + jj) * 16 + v) * 256 + t] = fmaf(cx[i][jj][v], inv, acc[i][jj][v]);
}

// Second kernel of the balanced schedule: the tiles of the super-tiles cut at XCD boundaries,
// head piece + tail piece, then the epilogue; one workgroup per tile and column block of 32
// (workgroup 4 (32 (xb - 1) + j) + i: cut xb, tile j, block i), so that the work spreads over
// every CU with few registers per thread.
template <int MODE, typename TT, int I>
__device__ __forceinline__ void split_fix_block(const float *p0, const float *p1, int r, int c, int M, int cols,
                                                const SplitEpi &e, unsigned char *gsm) {
  const int t = threadIdx.x;
  f16v acc[NB][MB], cx[NB][MB];
#pragma unroll
  for (int jj = 0; jj < MB; jj++) {
    cx[I][jj] = f16v{};
#pragma unroll
    for (int v = 0; v < 16; v++) {
      const int64_t o = (int64_t)((I * MB + jj) * 16 + v) * 256 + t;
      acc[I][jj][v] = p0[o] + p1[o];
    }
  }
  split_epilogue<MODE, TT, I, I + 1>(acc, cx, r, c, M, cols, e, gsm);
}

template <int MODE, typename TT>
__global__ __launch_bounds__(256) void k_split_gemm_fix(int64_t kp, int M, int cols, const SplitEpi e) {
  __shared__ double sred[4 * (GN / 2) * 2];
  BalShape bs;
  (void)bal_shape(M, cols, kp, bs);
  const int i = blockIdx.x & 3, j = (blockIdx.x >> 2) & 31, xb = 1 + (int)(blockIdx.x >> 7);
  const int64_t gc = bal_cut(bs, xb);
  if (gc % bs.nq == 0) return;  // this cut falls between super-tiles
  const int rho = j / bs.ctiles, c = j % bs.ctiles;
  if (rho >= bs.rps) return;
  const int r = (int)(gc / bs.nq) * bs.rps + rho;
  if (r >= bs.mtiles) return;
  const float *p0 = bal_slot(e.ws, xb, 0, j), *p1 = bal_slot(e.ws, xb, 1, j);
  unsigned char *gsm = (unsigned char *)sred;
  switch (i) {
    case 0: split_fix_block<MODE, TT, 0>(p0, p1, r, c, M, cols, e, gsm); break;
    case 1: split_fix_block<MODE, TT, 1>(p0, p1, r, c, M, cols, e, gsm); break;
    case 2: split_fix_block<MODE, TT, 2>(p0, p1, r, c, M, cols, e, gsm); break;
    default: split_fix_block<MODE, TT, 3>(p0, p1, r, c, M, cols, e, gsm); break;
  }
}

constexpr size_t split_gemm_lds() { return (size_t)3 * STAGE * sizeof(_Float16); }

template <int MODE, typename TT>
static hipError_t launch_mode(const void *st_h, const void *st_l, const void *m_h, const void *m_l, int64_t kp, int M,
                              int cols, const SplitEpi &e, hipStream_t s) {
  BalShape bs;
  if (bal_shape(M, cols, kp, bs)) {
    if (!e.ws) return hipErrorInvalidValue;
    k_split_gemm_bal<MODE, TT><<<8 * 32 * bal_pmax(bs), 256, split_gemm_lds(), s>>>((const _Float16 *)st_h, (const _Float16 *)st_l,
                                                                  (const _Float16 *)m_h, (const _Float16 *)m_l, kp, M,
                                                                  cols, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_split_gemm_fix<MODE, TT><<<7 * 32 * NB, 256, 0, s>>>(kp, M, cols, e);
    return hipGetLastError();
  }
  const int mtiles = (M + GM - 1) / GM, ctiles = (cols + GN - 1) / GN;
  const dim3 grid((unsigned)(8 * ((mtiles + 7) / 8) * ctiles));
  k_split_gemm<MODE, TT><<<grid, 256, split_gemm_lds(), s>>>((const _Float16 *)st_h, (const _Float16 *)st_l,
                                                             (const _Float16 *)m_h, (const _Float16 *)m_l, kp, M, cols, e);
  return hipGetLastError();
}

size_t split_gemm_ws_bytes(int M, int cols, int64_t kp) {
  BalShape bs;
  if (M <= 0 || cols <= 0 || kp <= 0 || !bal_shape(M, cols, kp, bs)) return 0;
  return (size_t)7 * 2 * 32 * BAL_SLOT * sizeof(float);
}

hipError_t launch_split_gemm_epi(int mode, const void *st_h, const void *st_l, const void *m_h, const void *m_l,
                                 int64_t kp, int M, int cols, const SplitEpi &e, hipStream_t s) {
  if (kp % SPLIT_KQUANT != 0 || kp <= 0 || M <= 0 || cols <= 0 || (cols & 1)) return hipErrorInvalidValue;
  const bool u16 = e.tbytes == 2;
  switch (mode) {
    case SE_PLAIN: return launch_mode<SE_PLAIN, uint8_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s);
    case SE_EIG: return launch_mode<SE_EIG, uint8_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s);
    case SE_REIG: return launch_mode<SE_REIG, uint8_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s);
    case SE_PHASE:
      return u16 ? launch_mode<SE_PHASE, uint16_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s)
                 : launch_mode<SE_PHASE, uint8_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s);
    case SE_LAST:
      return u16 ? launch_mode<SE_LAST, uint16_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s)
                 : launch_mode<SE_LAST, uint8_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s);
    case SE_RPHASE:
      return u16 ? launch_mode<SE_RPHASE, uint16_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s)
                 : launch_mode<SE_RPHASE, uint8_t>(st_h, st_l, m_h, m_l, kp, M, cols, e, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qaoa
