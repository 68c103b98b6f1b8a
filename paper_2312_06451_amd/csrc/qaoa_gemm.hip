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
// Tiling (gfx950, v_mfma_f32_32x32x16_f16): a workgroup of 256 threads owns a 128 x 128 tile
// of C^T (128 state columns x 128 rows of C), each wave a 64 x 64 quarter (2 x 2 blocks of 32
// x 32). The MFMA's first operand is the state (K-contiguous per column), the second the
// matrix (K-contiguous per row of op(V)), so the accumulator of a lane holds 4 consecutive
// rows of C per group and lanes run over consecutive rows: stores are 128-byte runs per
// column, and the real and imaginary columns of an angle set (adjacent columns) sit in the
// same lane. K advances in tiles of 32 through two LDS buffers: the next tile streams from
// global memory straight into one buffer (global_load_lds, 16 bytes per lane) while the
// current one is multiplied out of the other.
//
// Operand layout (blocked): each FP16 plane is stored as blocks of 128 rows x 32 halves, one
// per (row tile, K tile), K tiles of a row tile consecutive, rows inside a block in the
// chunk-swizzled order the LDS reads want; a K tile of a plane is therefore one contiguous
// 8 KB copy. Operands are zero-padded so every access is in bounds and unguarded: the matrix
// planes hold Mp = roundup(N, 128) rows of Kp = roundup(N, 32) halves, the state planes
// Ncp = roundup(cols, 128) columns of Kp halves. Every tile configuration is fixed at build
// time, so results do not depend on the process or the run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qaoa_internal.h"

namespace qaoa {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int GT = SPLIT_TILE;           // tile edge (rows of C, state columns)
constexpr int GK = SPLIT_KTILE;          // K tile
constexpr int BLK = GT * GK;             // halves per block (one plane, one tile, one K tile)
constexpr int BUF = 4 * BLK;             // halves per LDS buffer (four planes)

// Chunk swizzle of a block: row r holds its four 16-byte chunks in the order c ^ ((r >> 2) & 3),
// so the 16-byte fragment reads of 16 consecutive rows hit 64 distinct banks.
__device__ __forceinline__ int swz(int r, int c) { return c ^ ((r >> 2) & 3); }

// Thread-block loads of one K tile: wave w copies plane w (8 KB contiguous) into LDS, 1 KB per
// instruction, straight from global memory to LDS (no registers in between).
__device__ __forceinline__ void issue_tile(const _Float16 *const (&pl)[4], int kt, _Float16 *buf, int t) {
  const int lane = t & 63, w = t >> 6;
  const _Float16 *src = pl[w] + (int64_t)kt * BLK;
  _Float16 *dst = buf + w * BLK;
#pragma unroll
  for (int i = 0; i < 8; i++)
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(src + 512 * i + 8 * lane),
                                     (void __attribute__((address_space(3))) *)(dst + 512 * i), 16, 0, 0);
}

// The eight MFMA operand fragments of one 16-deep step: state hi/lo and matrix hi/lo of the
// wave's two 32-row blocks each (lane l: row l % 32, halves 8 (l / 32) .. + 7 of the step).
struct Frags {
  h8 ah[2], al[2], bh[2], bl[2];
};

__device__ __forceinline__ h8 frag(const _Float16 *buf, int plane, int r, int k) {
  return *(const h8 *)(buf + plane * BLK + r * GK + 8 * swz(r, k >> 3));
}

__device__ __forceinline__ void load_frags(Frags &f, const _Float16 *buf, int wn, int wm, int fr, int k) {
#pragma unroll
  for (int i = 0; i < 2; i++) {
    f.ah[i] = frag(buf, 0, wn + 32 * i + fr, k);
    f.al[i] = frag(buf, 1, wn + 32 * i + fr, k);
    f.bh[i] = frag(buf, 2, wm + 32 * i + fr, k);
    f.bl[i] = frag(buf, 3, wm + 32 * i + fr, k);
  }
}

__device__ __forceinline__ void mfma_step(const Frags &f, f16v (&acc)[2][2], f16v (&cx)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.ah[i], f.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) cx[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.al[i], f.bh[j], cx[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) cx[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.ah[i], f.bl[j], cx[i][j], 0, 0, 0);
}

}  // namespace

// acc (per lane: 2 x 2 blocks of 16 floats) of this workgroup's tile, = op(V) Psi; the
// epilogue is the caller's. The hi x hi products and the two cross products go to separate
// accumulators (each summed at its own scale), joined as hh + 2^-11 x at the end. Two LDS
// buffers: tile kt + 1 streams into one while tile kt is multiplied out of the other, one
// barrier per K tile.
__device__ __forceinline__ void split_gemm_tile(const _Float16 *__restrict__ st_h, const _Float16 *__restrict__ st_l,
                                                const _Float16 *__restrict__ m_h, const _Float16 *__restrict__ m_l,
                                                int64_t kp, int ct, int rt, _Float16 *lds, f16v (&acc)[2][2]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wn = (w >> 1) * 64, wm = (w & 1) * 64;  // this wave's state columns / rows of C
  const int nk = (int)(kp / GK);
  const _Float16 *const pl[4] = {st_h + (int64_t)ct * nk * BLK, st_l + (int64_t)ct * nk * BLK,
                                 m_h + (int64_t)rt * nk * BLK, m_l + (int64_t)rt * nk * BLK};
  f16v cx[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) {
      acc[i][j] = f16v{};
      cx[i][j] = f16v{};
    }
  const int fr = lane & 31, fk = 8 * (lane >> 5);
  issue_tile(pl, 0, lds, t);
  for (int kt = 0; kt < nk; kt++) {
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // this wave's loads of tile kt (vmcnt 0)
    __syncthreads();                                   // everyone's; everyone is done with tile kt - 1
    if (kt + 1 < nk) issue_tile(pl, kt + 1, lds + ((kt + 1) & 1) * BUF, t);
    const _Float16 *buf = lds + (kt & 1) * BUF;
    Frags f[2];
    load_frags(f[0], buf, wn, wm, fr, fk);
    load_frags(f[1], buf, wn, wm, fr, 16 + fk);
    mfma_step(f[0], acc, cx);
    mfma_step(f[1], acc, cx);
  }
  const float inv = 1.0f / 2048.0f;
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] += cx[i][j] * inv;
}

template <typename TT>
__device__ __forceinline__ uint32_t tab_at(const void *t, int64_t x) {
  return (uint32_t)((const TT *)t)[x];
}

// Sum v over the 32 rows of this lane's half-wave (lanes with the same lane >> 5), in a fixed
// butterfly order; every lane of the half ends with the sum.
__device__ __forceinline__ double rows_sum(double v) {
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// The product of one workgroup tile with epilogue MODE. Workgroup b runs on XCD b % 8
// (round-robin dispatch); each XCD takes the row tiles r = x (mod 8) and, for each, every
// column tile in consecutive workgroups, so the workgroups resident on one XCD at a time cover
// 8 row tiles x 8 column tiles and read each operand block once from memory into that XCD's L2.
template <int MODE, typename TT>
__global__ __launch_bounds__(256, 2) void k_split_gemm(const _Float16 *__restrict__ st_h,
                                                       const _Float16 *__restrict__ st_l,
                                                       const _Float16 *__restrict__ m_h,
                                                       const _Float16 *__restrict__ m_l, int64_t kp, int M,
                                                       int cols, const SplitEpi e) {
  extern __shared__ __align__(16) unsigned char gsm[];
  _Float16 *lds = (_Float16 *)gsm;
  const int ctiles = (cols + GT - 1) / GT, mtiles = (M + GT - 1) / GT;
  const int b = blockIdx.x, x = b & 7, j = b >> 3;
  const int r = 8 * (j / ctiles) + x, c = j % ctiles;
  if (r >= mtiles) return;
  f16v acc[2][2];
  split_gemm_tile(st_h, st_l, m_h, m_l, kp, c, r, lds, acc);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = r * GT + (w & 1) * 64, n0 = c * GT + (w >> 1) * 64;
  constexpr bool RED = MODE == SE_LAST || MODE == SE_REIG || MODE == SE_RPHASE;
  double red0[2][4][2], red1[2][4][2];  // per (column block, group, pair): this lane's row sums
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int g = 0; g < 4; g++)
#pragma unroll
      for (int h = 0; h < 2; h++) red0[i][g][h] = red1[i][g][h] = 0.0;
#pragma unroll
  for (int jj = 0; jj < 2; jj++) {
    const int m = m0 + 32 * jj + (lane & 31);
    if (m >= M) continue;
    double d = 0.0, cv = 0.0;
    uint32_t ci = 0;
    if constexpr (MODE == SE_EIG || MODE == SE_REIG) d = e.D[m];
    if constexpr (MODE == SE_PHASE || MODE == SE_LAST || MODE == SE_RPHASE) {
      ci = tab_at<TT>(e.table, m);
      cv = e.vals[ci];
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int g = 0; g < 4; g++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int n = n0 + 32 * i + 8 * g + 4 * (lane >> 5) + 2 * h;  // real-part column, even
          if (n >= cols) continue;
          const int sidx = n >> 1;
          float re = acc[i][jj][4 * g + 2 * h], im = acc[i][jj][4 * g + 2 * h + 1];
          if constexpr (MODE == SE_PLAIN) {
            e.C[m + (int64_t)n * e.ldc] = re;
            e.C[m + (int64_t)(n + 1) * e.ldc] = im;
            continue;
          }
          if constexpr (MODE == SE_REIG) {
            const float ta = e.ckr[m + (int64_t)n * e.ldc], tb = e.ckr[m + (int64_t)(n + 1) * e.ldc];
            red0[i][g][h] += d * ((double)re * tb - (double)im * ta);
          }
          if constexpr (MODE == SE_RPHASE) {
            const float pa = e.ckr[m + (int64_t)n * e.ldc], pb = e.ckr[m + (int64_t)(n + 1) * e.ldc];
            red0[i][g][h] += (cv - e.c0) * ((double)re * pb - (double)im * pa);
          }
          if constexpr (MODE == SE_LAST) {
            const double pr = (double)re * re + (double)im * im;
            red0[i][g][h] += pr * cv;
            red1[i][g][h] += pr;
            e.C[m + (int64_t)n * e.ldc] = re;
            e.C[m + (int64_t)(n + 1) * e.ldc] = im;
            if (e.bout) {
              const float k = (float)(cv - e.c0);
              split_emit(e.bout, e.bld, e.bplane, m, sidx, k * re, k * im);
            }
            continue;
          }
          if constexpr (MODE == SE_EIG || MODE == SE_REIG) {
            double sn, cs;
            sincos((MODE == SE_EIG ? -1.0 : 1.0) * e.betas[sidx] * d, &sn, &cs);
            const float a = re, bb = im;
            re = (float)((double)a * cs - (double)bb * sn);
            im = (float)((double)a * sn + (double)bb * cs);
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
    // rows of this wave -> lanes 0 and 32; the two waves of a column half meet in LDS, in order
    __syncthreads();  // every wave is done with the last K tile in LDS
    double *sred = (double *)gsm;  // [wave][32 sets][2]
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int g = 0; g < 4; g++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const double s0 = rows_sum(red0[i][g][h]);
          const double s1 = MODE == SE_LAST ? rows_sum(red1[i][g][h]) : 0.0;
          if ((lane & 31) == 0) {
            const int sl = (32 * i + 8 * g + 4 * (lane >> 5) + 2 * h) >> 1;  // set within the wave's 64 columns
            sred[(w * 32 + sl) * 2] = s0;
            sred[(w * 32 + sl) * 2 + 1] = s1;
          }
        }
    __syncthreads();
    if (t < 64) {
      const int half = t >> 5, sl = t & 31;  // column half (wn) and set within it
      const int wa = 2 * half, wb = 2 * half + 1;  // the waves with rows 0..63 and 64..127
      const int s = (c * GT + 64 * half) / 2 + sl;
      if (2 * s < cols) {
        const double a0 = sred[(wa * 32 + sl) * 2] + sred[(wb * 32 + sl) * 2];
        e.part0[(int64_t)s * e.nblk + r] = a0;
        if (MODE == SE_LAST) e.part1[(int64_t)s * e.nblk + r] = sred[(wa * 32 + sl) * 2 + 1] + sred[(wb * 32 + sl) * 2 + 1];
      }
    }
  }
}

constexpr size_t split_gemm_lds() { return (size_t)2 * BUF * sizeof(_Float16); }

template <int MODE, typename TT>
static hipError_t launch_mode(const void *st_h, const void *st_l, const void *m_h, const void *m_l, int64_t kp, int M,
                              int cols, const SplitEpi &e, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t er = hipFuncSetAttribute((const void *)k_split_gemm<MODE, TT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)split_gemm_lds());
    if (er != hipSuccess) return er;
    attr_set = true;
  }
  const int mtiles = (M + GT - 1) / GT, ctiles = (cols + GT - 1) / GT;
  const dim3 grid((unsigned)(8 * ((mtiles + 7) / 8) * ctiles));
  k_split_gemm<MODE, TT><<<grid, 256, split_gemm_lds(), s>>>((const _Float16 *)st_h, (const _Float16 *)st_l,
                                                             (const _Float16 *)m_h, (const _Float16 *)m_l, kp, M, cols, e);
  return hipGetLastError();
}

hipError_t launch_split_gemm_epi(int mode, const void *st_h, const void *st_l, const void *m_h, const void *m_l,
                                 int64_t kp, int M, int cols, const SplitEpi &e, hipStream_t s) {
  if (kp % GK != 0 || M <= 0 || cols <= 0 || (cols & 1)) return hipErrorInvalidValue;
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

hipError_t launch_split_gemm(const void *st_h, const void *st_l, const void *m_h, const void *m_l, int64_t kp,
                             int M, int cols, float *C, int64_t ldc, hipStream_t s) {
  SplitEpi e{};
  e.C = C;
  e.ldc = ldc;
  e.tbytes = 1;
  return launch_split_gemm_epi(SE_PLAIN, st_h, st_l, m_h, m_l, kp, M, cols, e, s);
}

}  // namespace qaoa
