// HIP kernels for gfx950 (MI355X): QAOA statevector evolution with the transverse-field
// mixer (Golden et al., JuliQAOA, SC-W 2023).
//
//  (a) cost table C(x) over the feasible set (Sec. 2.1, pre-computation);
//  (b) phase separator e^{-i gamma C(x)} as a lookup-table multiply (Eq. (1));
//  (c) mixer e^{-i beta sum_q X_q} as one 2x2 rotation per qubit (the factorisation of
//      Eq. (2));
//  (d) <C> = sum_x |psi(x)|^2 C(x) (Sec. 1) and the gradient in (beta, gamma) by a reverse
//      sweep that undoes each layer (Sec. 2.3 gets this gradient by reverse-mode AD).
//
// Rotation form. A qubit rotation e^{-i b X} = cos b I - i sin b X is applied unnormalised as
// G(tau) = I - i tau X (four FMAs per amplitude pair) with tau = tan b, or, when |tan b| > 1,
// as X G(tau) with tau = -cot b. The dropped scalar (cos b, or -i sin b) is tracked by the
// host and folded into the next phase lookup table, so every applied rotation is exactly
// unitary up to that scalar and norm drift does not accumulate. The X of the second form is
// not applied either: the stored vector is the state with a known set of bits flipped
// (after a full round: all bits or none, so at every phase point). Steps that read the cost
// then read C(~x): tables with C(~x) = C(x) (every MaxCut table) are read unchanged, other
// tables through their reversed copy, chosen per angle set; a state export un-flips.
//
// Cost tables hold, per state, the index of its value among at most 1024 distinct values;
// the phase lookup tables and a small value table (staged in LDS) map indices to
// e^{-i gamma c} and to c.
//
// Tile passes. A workgroup of 256 threads holds a tile of 2^T amplitudes in registers
// (2^(T-8) per thread and vector). Tile bits [0,c) are contiguous address bits; the other
// T-c tile bits sit on a contiguous range of higher address bits. Rotations on tile bits that
// live in a thread's registers need no communication; three register assignments (H, M, L)
// cover all tile bits and the tile moves between them through a padded, bank-conflict-free
// LDS buffer. The phase multiply, the <C> reduction, the adjoint initialisation and the
// gradient inner products are fused into the passes.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>
#include <vector>
#include <cstdint>
#include "qaoa_internal.h"

namespace qaoa {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T2 = float2; };
template <> struct Cplx<double> { using T2 = double2; };

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Materialise a partial sum where it is computed. The sums only feed the final reduction, so
// without this the compiler sinks their arithmetic to the end of the kernel and keeps the
// amplitudes they read alive across every later stage.
__device__ __forceinline__ void pin(float &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

// A workgroup-uniform 64-bit value, pinned to scalar registers (so global accesses take the
// SGPR-base + 32-bit VGPR-offset form).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
// A uniform value the compiler must treat as new: values derived from it are recomputed
// rather than kept live (in scalar registers, or spilled to vector lanes) from an earlier use.
__device__ __forceinline__ uint32_t fresh_s(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// ============================================================== (a) cost table

// C(x) = sum_e w_e [bit u_e of x != bit v_e of x], one x per thread (grid-stride, 64-bit x).
template <typename TT>
__global__ void k_cost_table_full(int n, int m, const int32_t *__restrict__ u,
                                  const int32_t *__restrict__ v, const int32_t *__restrict__ w,
                                  TT *__restrict__ table) {
  __shared__ int32_t su[512], sv[512], sw[512];
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    su[e] = u[e];
    sv[e] = v[e];
    sw[e] = w ? w[e] : 1;
  }
  __syncthreads();
  const uint64_t N = 1ull << n;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
    uint32_t c = 0;
    for (int e = 0; e < m; e++) c += (uint32_t)sw[e] * (uint32_t)(((x >> su[e]) ^ (x >> sv[e])) & 1u);
    table[x] = (TT)c;
  }
}

// Weight-k feasible set: the r-th weight-k integer in increasing order, found by the
// combinatorial number system (largest a with C(a, i) <= r, for i = k..1).
template <typename TT>
__global__ void k_cost_table_hw(int n, int k, int m, const int32_t *__restrict__ u,
                                const int32_t *__restrict__ v, const int32_t *__restrict__ w,
                                const int64_t *__restrict__ binom, uint64_t N,
                                TT *__restrict__ table) {
  __shared__ int32_t su[512], sv[512], sw[512];
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    su[e] = u[e];
    sv[e] = v[e];
    sw[e] = w ? w[e] : 1;
  }
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += stride) {
    uint64_t rem = r, x = 0;
    int a = n - 1;
    for (int i = k; i >= 1; i--) {
      while (a >= i && (uint64_t)binom[a * 33 + i] > rem) a--;
      x |= 1ull << a;
      rem -= (uint64_t)binom[a * 33 + i];
      a--;
    }
    uint32_t c = 0;
    for (int e = 0; e < m; e++) c += (uint32_t)sw[e] * (uint32_t)(((x >> su[e]) ^ (x >> sv[e])) & 1u);
    table[r] = (TT)c;
  }
}

template <typename TT>
__global__ void k_table_max(const TT *__restrict__ t, uint64_t N, unsigned *__restrict__ out) {
  unsigned mx = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    mx = max(mx, (unsigned)t[i]);
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (unsigned)__shfl_xor((int)mx, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, mx);
}

// dst[r * 2^T + e] = src[address(r, e)] for the tile geometry (T, c, h0).
template <typename TT>
__global__ void k_table_relayout(const TT *__restrict__ src, TT *__restrict__ dst, int n, int T,
                                 int c, int h0) {
  const uint64_t N = 1ull << n;
  const int lo_w = h0 - c;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    uint64_t r = i >> T, e = i & ((1ull << T) - 1);
    uint64_t x = ((r & ((1ull << lo_w) - 1)) << c) | ((r >> lo_w) << (h0 + T - c)) |
                 (e & ((1ull << c) - 1)) | ((e >> c) << h0);
    dst[i] = src[x];
  }
}

template <typename TT>
__global__ void k_table_widen(const TT *__restrict__ src, int64_t *__restrict__ dst, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    dst[i] = (int64_t)src[i];
}

// dst[i] = src[N - 1 - i]: the table of C(~x) over the full space, in any tile-major layout
// (complementing x complements both the tile index and the element index).
template <typename TT>
__global__ void k_table_reverse(const TT *__restrict__ src, TT *__restrict__ dst, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    dst[i] = src[N - 1 - i];
}

template <typename TT>
__global__ void k_table_values(const TT *__restrict__ src, const double *__restrict__ vals,
                               double *__restrict__ dst, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    dst[i] = vals[src[i]];
}

// ============================================================== phase lookup tables

// luts[j][c] = s_j * exp(sign_j * i * gamma_j * vals[c]): FP64 argument and sincos, one
// rounding.
template <typename R>
__global__ void k_luts(const LutJob *__restrict__ jobs, int lut_len, const double *__restrict__ vals,
                       typename Cplx<R>::T2 *__restrict__ luts) {
  const LutJob J = jobs[blockIdx.x];
  for (int c = threadIdx.x; c < lut_len; c += blockDim.x) {
    double s, co;
    sincos(J.sign * J.gamma * vals[c], &s, &co);
    typename Cplx<R>::T2 o;
    o.x = (R)(J.sre * co - J.sim * s);
    o.y = (R)(J.sre * s + J.sim * co);
    luts[(size_t)blockIdx.x * lut_len + c] = o;
  }
}

// ============================================================== tile passes

enum { AH = 0, AM = 1, AL = 2 };

template <int T>
struct TileCfg {
  static constexpr int TB = 8;                 // thread bits (256 threads)
  static constexpr int RB = T - TB;            // register bits per thread
  static constexpr int RN = 1 << RB;           // amplitudes per thread per vector
  static constexpr int MLO = T - 2 * RB;       // assignment M holds tile bits [MLO, MLO+RB)
  static_assert(MLO >= 0 && 3 * RB >= T, "tile shape");
  static_assert(((1u << T) / 16) % 256 == 0, "table tile: whole 16-byte chunks per thread");
};

// Tile index of register j of thread t in assignment A.
template <int A, int T>
__device__ __forceinline__ uint32_t elem(uint32_t t, uint32_t j) {
  using G = TileCfg<T>;
  if constexpr (A == AH) return t | (j << G::TB);
  else if constexpr (A == AM)
    return (t & ((1u << G::MLO) - 1)) | (j << G::MLO) | ((t >> G::MLO) << (G::MLO + G::RB));
  else return j | (t << G::RB);
}
// Tile bit held by register bit b in assignment A.
template <int A, int T>
__device__ constexpr int regbit(int b) {
  using G = TileCfg<T>;
  return A == AH ? G::TB + b : (A == AM ? G::MLO + b : b);
}
// Tile bits rotated while in assignment A: H owns [TB,T), M owns [RB,TB), L owns [0,RB).
template <int A, int T>
__device__ constexpr uint32_t group(void) {
  using G = TileCfg<T>;
  return A == AH ? (((1u << T) - 1) & ~((1u << G::TB) - 1))
                 : (A == AM ? (((1u << G::TB) - 1) & ~((1u << G::RB) - 1)) : ((1u << G::RB) - 1));
}

// Padded LDS layout: tile element e sits in slot e + (e >> PS), one pad slot per 256 bytes
// (PS = 5 for complex64, 4 for complex128); conflict-free in all three assignments. For
// every assignment the slot splits into a per-thread base plus a constant per register.
template <typename R> struct Pad { static constexpr int PS = sizeof(R) == 4 ? 5 : 4; };

template <typename R, int T, int A>
__device__ __forceinline__ uint32_t lbase(uint32_t t) {
  using G = TileCfg<T>;
  constexpr int PS = Pad<R>::PS;
  if constexpr (A == AH) return t + (t >> PS);
  else if constexpr (A == AM)
    return (t & ((1u << G::MLO) - 1)) +
           (t >> G::MLO) * ((1u << (G::MLO + G::RB)) + (1u << (G::MLO + G::RB - PS)));
  else return (t << G::RB) + ((t << G::RB) >> PS);  // register part below bit PS: no carry
}
template <typename R, int T, int A>
__device__ constexpr uint32_t loff(int j) {
  using G = TileCfg<T>;
  constexpr int PS = Pad<R>::PS;
  if constexpr (A == AH) return (uint32_t)j * ((1u << G::TB) + (1u << (G::TB - PS)));
  else if constexpr (A == AM) return ((uint32_t)j << G::MLO) + (((uint32_t)j << G::MLO) >> PS);
  else return (uint32_t)j + ((uint32_t)j >> PS);
}

// Staged table: byte position of entry e is e*s + 16 * ((e*s) >> 8) (s = entry size); per
// assignment again a per-thread base plus a constant per register.
template <int T, int A, int S>
__device__ __forceinline__ uint32_t tbase(uint32_t t) {
  using G = TileCfg<T>;
  // e(t, 0) * S, then padding; valid because the register part never carries into the
  // thread part across a 256-byte boundary in any assignment
  uint32_t e0;
  if constexpr (A == AH) e0 = t;
  else if constexpr (A == AM) e0 = (t & ((1u << G::MLO) - 1)) | ((t >> G::MLO) << (G::MLO + G::RB));
  else e0 = t << G::RB;
  return e0 * S + (((e0 * S) >> 8) << 4);
}
template <int T, int A, int S>
__device__ constexpr uint32_t toffc(int j) {
  using G = TileCfg<T>;
  uint32_t ej = A == AH ? ((uint32_t)j << G::TB) : (A == AM ? ((uint32_t)j << G::MLO) : (uint32_t)j);
  return ej * S + (((ej * S) >> 8) << 4);
}

template <typename R, int T, int A>
__device__ __forceinline__ void to_lds(typename Cplx<R>::T2 *lds, const typename Cplx<R>::T2 *v,
                                       uint32_t t) {
  typename Cplx<R>::T2 *p = lds + lbase<R, T, A>(t);
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) p[loff<R, T, A>(j)] = v[j];
}
template <typename R, int T, int A>
__device__ __forceinline__ void from_lds(const typename Cplx<R>::T2 *lds,
                                         typename Cplx<R>::T2 *v, uint32_t t) {
  const typename Cplx<R>::T2 *p = lds + lbase<R, T, A>(t);
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) v[j] = p[loff<R, T, A>(j)];
}

// Move one vector from assignment FROM to assignment TO through LDS.
template <typename R, int T, int FROM, int TO>
__device__ __forceinline__ void xchg1(typename Cplx<R>::T2 *lds, typename Cplx<R>::T2 *v,
                                      uint32_t t) {
  __syncthreads();
  to_lds<R, T, FROM>(lds, v, t);
  __syncthreads();
  from_lds<R, T, TO>(lds, v, t);
}

// Exchange through a half-size buffer in two rounds, split on tile bit T - 1 (register bit
// RB - 1 in assignment H, thread bit 7 in M and L): round h moves the amplitudes whose tile
// bit T - 1 is h. A thread that must read before it has written all of its own registers
// parks the values in `tmp` (register-to-thread moves at h = 0), or all threads read the
// first half into `tmp` (thread-to-register moves), so nothing is overwritten unsent.
template <typename R, int T, int FROM, int TO, int HB>
__device__ __forceinline__ void xchgh_round(typename Cplx<R>::T2 *lds, typename Cplx<R>::T2 *v,
                                            typename Cplx<R>::T2 *tmp, uint32_t t, uint32_t tb) {
  using G = TileCfg<T>;
  constexpr int RN = G::RN, HN = RN / 2;
  constexpr uint32_t D = HB ? (1u << (T - 1)) + (1u << (T - 1 - Pad<R>::PS)) : 0u;  // slots of the lower half
  __syncthreads();
  typename Cplx<R>::T2 *pf = lds + lbase<R, T, FROM>(t) - D;
  if constexpr (FROM == AH) {
#pragma unroll
    for (int j = 0; j < RN; j++)
      if (((j >> (G::RB - 1)) & 1) == HB) pf[loff<R, T, FROM>(j)] = v[j];
  } else {
    if (tb == (uint32_t)HB) {
#pragma unroll
      for (int j = 0; j < RN; j++) pf[loff<R, T, FROM>(j)] = v[j];
    }
  }
  __syncthreads();
  const typename Cplx<R>::T2 *pt = lds + lbase<R, T, TO>(t) - D;
  if constexpr (TO == AH) {
#pragma unroll
    for (int j = 0; j < RN; j++)
      if (((j >> (G::RB - 1)) & 1) == HB) {
        if (HB == 0) tmp[j] = pt[loff<R, T, TO>(j)];
        else v[j] = pt[loff<R, T, TO>(j)];
      }
  } else {
    if (tb == (uint32_t)HB) {
#pragma unroll
      for (int j = 0; j < RN; j++) {
        if (FROM == AH && HB == 0 && j >= HN) tmp[j - HN] = pt[loff<R, T, TO>(j)];
        else v[j] = pt[loff<R, T, TO>(j)];
      }
    }
  }
}
template <typename R, int T, int FROM, int TO>
__device__ __forceinline__ void xchg1h(typename Cplx<R>::T2 *lds, typename Cplx<R>::T2 *v, uint32_t t) {
  if constexpr (FROM != TO) {
    using G = TileCfg<T>;
    constexpr int HN = G::RN / 2;
    typename Cplx<R>::T2 tmp[HN];
    const uint32_t tb = (t >> 7) & 1u;  // tile bit T - 1 in assignments M and L
    xchgh_round<R, T, FROM, TO, 0>(lds, v, tmp, t, tb);
    xchgh_round<R, T, FROM, TO, 1>(lds, v, tmp, t, tb);
    if constexpr (TO == AH) {
#pragma unroll
      for (int j = 0; j < HN; j++) v[j] = tmp[j];
    } else if constexpr (FROM == AH) {
      if (tb == 0) {
#pragma unroll
        for (int j = 0; j < HN; j++) v[HN + j] = tmp[j];
      }
    }
  }
}

// (a, b) <- (a - i tau b, b - i tau a)
template <typename T2, typename R>
__device__ __forceinline__ void bfly(T2 &a, T2 &b, R tau) {
  T2 na, nb;
  na.x = fmaR(tau, b.y, a.x);
  na.y = fmaR(-tau, b.x, a.y);
  nb.x = fmaR(tau, a.y, b.x);
  nb.y = fmaR(-tau, a.x, b.y);
  a = na;
  b = nb;
}
// Im(conj(la) pb + conj(lb) pa): the X-pair term of one amplitude pair.
template <typename T2, typename R>
__device__ __forceinline__ R xpair(const T2 &pa, const T2 &pb, const T2 &la, const T2 &lb, R acc) {
  acc = fmaR(la.x, pb.y, acc);
  acc = fmaR(-la.y, pb.x, acc);
  acc = fmaR(lb.x, pa.y, acc);
  acc = fmaR(-lb.y, pa.x, acc);
  return acc;
}

// X-pair terms of register bit B: sum over the thread's pairs of Im(conj(la) pb + conj(lb) pa),
// with two accumulators to shorten the dependency chain.
template <typename R, int T, int B>
__device__ __forceinline__ R xterm_bit(const typename Cplx<R>::T2 *phi, const typename Cplx<R>::T2 *lam) {
  using G = TileCfg<T>;
  R s0 = 0, s1 = 0;
  int k = 0;
#pragma unroll
  for (int j = 0; j < G::RN; j++) {
    if (j & (1 << B)) continue;
    if (k++ & 1) s1 = xpair(phi[j], phi[j | (1 << B)], lam[j], lam[j | (1 << B)], s1);
    else s0 = xpair(phi[j], phi[j | (1 << B)], lam[j], lam[j | (1 << B)], s0);
  }
  return s0 + s1;
}

// Rotation of register bit B (compile-time, so every register index is a constant and the
// arrays stay in VGPRs). A tile bit that is not rotated in this pass (a passenger) gets
// tau = 0, which FMA applies exactly as the identity: the stage is branch-free.
template <typename R, int T, int NV, int B, bool ROT_LAM>
__device__ __forceinline__ void rot_bit(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam, R tau) {
  using G = TileCfg<T>;
#pragma unroll
  for (int j = 0; j < G::RN; j++)
    if (!(j & (1 << B))) bfly(phi[j], phi[j | (1 << B)], tau);
  if constexpr (NV == 2 && ROT_LAM) {
#pragma unroll
    for (int j = 0; j < G::RN; j++)
      if (!(j & (1 << B))) bfly(lam[j], lam[j | (1 << B)], tau);
  }
  // keep the bit-by-bit (in-place) order: interleaving bits multiplies the live registers
  __builtin_amdgcn_sched_barrier(0);
}

// X-pair terms of the register bits B.. of assignment A that are rotated in this pass, all at
// the stage's starting point (they do not change under the rotations of the round, up to
// the tracked scalar), weighted with w.
template <typename R, int T, int A, int B>
__device__ __forceinline__ void xterms(const typename Cplx<R>::T2 *phi, const typename Cplx<R>::T2 *lam,
                                       uint32_t mask, double w, double &acc) {
  using G = TileCfg<T>;
  if constexpr (B < G::RB) {
    constexpr int tb = regbit<A, T>(B);
    if constexpr ((group<A, T>() >> tb) & 1u) {
      R sb = xterm_bit<R, T, B>(phi, lam);
      pin(sb);
      acc += (((mask >> tb) & 1u) ? w : 0.0) * (double)sb;
    }
    xterms<R, T, A, B + 1>(phi, lam, mask, w, acc);
  }
}

template <typename R, int T, int NV, int A, bool ROT_LAM, int B>
__device__ __forceinline__ void rot_bits(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                         uint32_t mask, R tau, double shrink, double &w) {
  using G = TileCfg<T>;
  if constexpr (B < G::RB) {
    constexpr int tb = regbit<A, T>(B);
    if constexpr ((group<A, T>() >> tb) & 1u) {
      const bool on = (mask >> tb) & 1u;  // uniform
      rot_bit<R, T, NV, B, ROT_LAM>(phi, lam, on ? tau : (R)0);
      if (on) w *= shrink;
    }
    rot_bits<R, T, NV, A, ROT_LAM, B + 1>(phi, lam, mask, tau, shrink, w);
  }
}

// One register stage: every register bit of assignment A whose tile bit belongs to A's group
// is processed; bits in `mask` are rotated (their X-pair terms taken first when XT), the
// others pass.
template <typename R, int T, int NV, int A, bool ROT_LAM, bool XT>
__device__ __forceinline__ void stage(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                      uint32_t mask, R tau, double &w, double &acc) {
  if constexpr (NV == 2 && XT) {
    xterms<R, T, A, 0>(phi, lam, mask, w, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
  const double shrink = 1.0 / (1.0 + (double)tau * (double)tau);
  rot_bits<R, T, NV, A, ROT_LAM, 0>(phi, lam, mask, tau, shrink, w);
}

// Staged table entry of register j (assignment A) of the thread whose base is tb.
template <typename TT, int T, int A>
__device__ __forceinline__ uint32_t tab_at(const unsigned char *tb, int j) {
  return (uint32_t)(*(const TT *)(tb + toffc<T, A, (int)sizeof(TT)>(j)));
}

template <typename T2, typename R>
__device__ __forceinline__ T2 cmul(const T2 &v, const T2 &L) {
  T2 o;
  o.x = fmaR(v.x, L.x, -v.y * L.y);
  o.y = fmaR(v.x, L.y, v.y * L.x);
  return o;
}

// Elementwise steps in assignment A, each step in its own loop (no per-element branching).
// MID != 0 fixes the steps at compile time (flag bits of the PF_ set); MID == 0 reads them
// from the pass flags.
template <typename R, int T, int NV, typename TT, int A, uint32_t MID>
__device__ __forceinline__ void middle(const PassArgs<R> &a, const SetParams<R> &sp,
                                       typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                       const unsigned char *ltab,
                                       const typename Cplx<R>::T2 *llut, const R *lval, uint32_t t,
                                       double w, double *acc) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  constexpr uint32_t f = MID;
  const unsigned char *tb = ltab + tbase<T, A, (int)sizeof(TT)>(t);
  if (f & PF_EXPECT) {
    R e_acc = 0, n_acc = 0;
#pragma unroll
    for (int j = 0; j < G::RN; j++) {
      const R cr = lval[tab_at<TT, T, A>(tb, j)];
      R pr = fmaR(phi[j].x, phi[j].x, phi[j].y * phi[j].y);
      e_acc = fmaR(pr, cr, e_acc);
      n_acc += pr;
    }
    pin(e_acc);
    pin(n_acc);
    acc[SL_A] += (double)e_acc;
    acc[SL_B] += (double)n_acc;
  }
  if constexpr (NV == 2) {
    if (f & PF_LAMBDA) {
#pragma unroll
      for (int j = 0; j < G::RN; j++) {
        const R cr = lval[tab_at<TT, T, A>(tb, j)];
        R kf = sp.lam_rho * (cr - a.lam_c0);
        lam[j].x = kf * phi[j].x;
        lam[j].y = kf * phi[j].y;
      }
    }
    if (f & PF_GGAMMA) {
      // Im <lam|C|phi> = Im <lam|(C - c0)|phi>: <lam|phi> = <psi_p|(C - c0)|psi_p> is real.
      // The centred form keeps the multiplier at the spread of C rather than its maximum,
      // and the products are summed in FP64.
      double g_acc = 0;
#pragma unroll
      for (int j = 0; j < G::RN; j++) {
        const R cr = lval[tab_at<TT, T, A>(tb, j)] - a.lam_c0;
        R im = fmaR(lam[j].x, phi[j].y, -lam[j].y * phi[j].x);
        g_acc += (double)(im * cr);
      }
      pin(g_acc);
      acc[SL_B] += w * g_acc;
    }
  }
  if (f & PF_PHASE) {
#pragma unroll
    for (int j = 0; j < G::RN; j++) {
      const T2 L = llut[tab_at<TT, T, A>(tb, j)];
      phi[j] = cmul<T2, R>(phi[j], L);
      if constexpr (NV == 2) lam[j] = cmul<T2, R>(lam[j], L);
    }
  }
}

// Move both vectors (NV of them) from assignment FROM to assignment TO (compile time).
template <typename R, int T, int NV, int FROM, int TO>
__device__ __forceinline__ void xchg(typename Cplx<R>::T2 *lds, typename Cplx<R>::T2 *phi,
                                     typename Cplx<R>::T2 *lam, uint32_t t) {
  if constexpr (FROM != TO) {
    xchg1<R, T, FROM, TO>(lds, phi, t);
    if constexpr (NV == 2) xchg1<R, T, FROM, TO>(lds, lam, t);
  }
}

// Tile passes over one vector that do more than one register block (or start a sweep) use
// the half-size exchange: half the LDS, so three workgroups fit on a CU and one workgroup's
// loads overlap another's stages. The single-block forward pass keeps the full exchange
// (fewer barriers; it already streams at the copy rate), and so do the two-vector passes
// (their registers would not leave room for three workgroups); passes whose stages stay in
// assignment H exchange nothing.
template <int KIND, int S1, int S2>
constexpr bool pass_half_xchg() { return KIND == 1 && !(S1 == 7 && S2 == 0) && ((S1 | S2) & 6) != 0; }

template <typename R, int T, int FROM, int TO, bool HALF>
__device__ __forceinline__ void xchg1p(typename Cplx<R>::T2 *lds, typename Cplx<R>::T2 *v, uint32_t t) {
  if constexpr (HALF) xchg1h<R, T, FROM, TO>(lds, v, t);
  else xchg1<R, T, FROM, TO>(lds, v, t);
}
template <typename R, int T, int NV, int FROM, int TO, bool HALF>
__device__ __forceinline__ void xchgp(typename Cplx<R>::T2 *lds, typename Cplx<R>::T2 *phi,
                                      typename Cplx<R>::T2 *lam, uint32_t t) {
  if constexpr (FROM != TO) {
    xchg1p<R, T, FROM, TO, HALF>(lds, phi, t);
    if constexpr (NV == 2) xchg1p<R, T, FROM, TO, HALF>(lds, lam, t);
  }
}

// Register assignment after the stages of set S (bit 0: H, bit 1: M, bit 2: L) visited in the
// order H, M, L (DOWN) or L, M, H (UP), starting from assignment START.
template <int S, bool DOWN, int START>
constexpr int after_stages() {
  if constexpr (DOWN) return (S & 4) ? AL : ((S & 2) ? AM : ((S & 1) ? AH : START));
  else return (S & 1) ? AH : ((S & 2) ? AM : ((S & 4) ? AL : START));
}

// One tile pass. KIND 1: forward over phi. KIND 2: reverse sweep over (phi, lam): part 1 undoes
// the forward pass's last rotation block (X-pair terms first), the middle reads the gamma
// gradient and undoes the phase, part 2 undoes the first block. KIND 4: KIND 2 reading phi
// from a forward checkpoint and never storing it, so the last stage's rotation of phi is dead
// code and compiled out. KIND 3: end of the forward sweep on phi (part 1), <C> and
// lam = rho (C - c0) phi (middle), then the reverse sweep's first block on both (part 2).
// S1 / S2: register stages of part 1 / part 2.
template <typename R, int T, int KIND, int S1, int S2, int SHAPE, typename TT>
__global__ __launch_bounds__(256, (pass_half_xchg<KIND, S1, S2>() ? 3 : 2)) void k_pass(const PassArgs<R> a) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  constexpr int NV = KIND == 1 ? 1 : 2;
  constexpr int RN = G::RN;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool HALF = pass_half_xchg<KIND, S1, S2>();
  constexpr uint32_t kStateSlots = ((1u << T) >> (HALF ? 1 : 0)) + (((1u << T) >> (HALF ? 1 : 0)) >> Pad<R>::PS);
  constexpr uint32_t kTabBytes = ((1u << T) * sizeof(TT)) + (((1u << T) * sizeof(TT)) >> 8) * 16;
  T2 *lds = (T2 *)smem;
  unsigned char *ltab = smem + kStateSlots * sizeof(T2);
  T2 *llut = (T2 *)(ltab + kTabBytes);
  R *lval = (R *)(llut + a.lut_len);
  double *lred = (double *)smem;  // reused after the last exchange

  const uint32_t t = threadIdx.x;
  const uint32_t b = blockIdx.x;
  const uint32_t q = blockIdx.y;  // angle set
  const uint32_t r = a.xcd_remap ? ((b & 7u) * (a.nwg >> 3) + (b >> 3)) : b;
  const SetParams<R> sp = a.sp[q];
  const uint32_t f = a.flags;

  const int lo_w = a.h0 - a.c;
  const uint64_t base = (((uint64_t)r & ((1ull << lo_w) - 1)) << a.c) |
                        (((uint64_t)r >> lo_w) << (a.h0 + T - a.c));
  const uint64_t cmask = (1ull << a.c) - 1;
  // element offset of tile index e (a bit deposit, additive over disjoint bits)
  auto off = [&](uint32_t e) -> uint64_t {
    return ((uint64_t)e & cmask) | (((uint64_t)e >> a.c) << a.h0);
  };
  // per-thread byte offset (32 bits suffice: the thread's tile bits stay below address bit
  // n - 3) and uniform per-register byte offsets
  const uint32_t tbyte = (uint32_t)(off(t) * sizeof(T2));
  auto jbyte = [&](int j) -> uint64_t { return off((uint32_t)j << G::TB) * sizeof(T2); };
  // element j of a vector whose (uniform) byte base is vb: a global-address-space pointer with
  // a scalar base and the thread's 32-bit byte offset
  using V2 = R __attribute__((ext_vector_type(2)));
  using gbyte = __attribute__((address_space(1))) unsigned char;
  using gV2 = __attribute__((address_space(1))) V2;
  auto at = [&](uint64_t vb, int j) -> gV2 * { return (gV2 *)((gbyte *)uniform64(vb + jbyte(j)) + tbyte); };
  auto ld = [&](uint64_t vb, int j) -> T2 { V2 v = *at(vb, j); return T2{v.x, v.y}; };
  // stores recompute the per-register offsets (from fresh copies of the geometry) instead of
  // keeping the loads' 32 64-bit offsets live across the whole pass
  auto st = [&](uint64_t vb, int j, const T2 &x) {
    const uint32_t cs = fresh_s((uint32_t)a.c), hs = fresh_s((uint32_t)a.h0);
    const uint64_t e = (uint64_t)j << G::TB;
    const uint64_t jb = ((e & ((1ull << cs) - 1)) | ((e >> cs) << hs)) * sizeof(T2);
    V2 v;
    v.x = x.x;
    v.y = x.y;
    *(gV2 *)((gbyte *)uniform64(vb + jb) + tbyte) = v;
  };
  const uint64_t vs = ((uint64_t)q * a.vstride + base) * sizeof(T2);

  T2 phi[RN];
  T2 lam[NV == 2 ? RN : 1];

  // ---- this tile's table bytes, loaded into registers ahead of the state so that writing
  // them to LDS later waits only for these loads
  constexpr bool need_tab = SHAPE != 0;
  constexpr uint32_t kTabChunks = need_tab ? ((1u << T) * sizeof(TT)) / 16 / 256 : 1;  // 16 B per thread each
  uint4 tpre[kTabChunks];
  if constexpr (need_tab) {
    const uint4 *tsrc = (const uint4 *)((const unsigned char *)(sp.tflip ? a.table_rev : a.table) +
                                        (uint64_t)r * ((1ull << T) * sizeof(TT)));
#pragma unroll
    for (uint32_t k = 0; k < kTabChunks; k++) tpre[k] = tsrc[t + 256 * k];
  }
  // ---- load (assignment H: lanes run over contiguous address bits)
  {
    const uint64_t src = (f & PF_LOAD_PSI0) ? (uint64_t)a.psi0 + base * sizeof(T2) : (uint64_t)a.phi + vs;
    if (f & (PF_LOAD_PHI | PF_LOAD_PSI0)) {
#pragma unroll
      for (int j = 0; j < RN; j++) phi[j] = ld(src, j);
      if (f & PF_LOAD_SCALE) {
        const T2 k{sp.out_re, sp.out_im};
#pragma unroll
        for (int j = 0; j < RN; j++) phi[j] = cmul<T2, R>(phi[j], k);
      }
    } else {
#pragma unroll
      for (int j = 0; j < RN; j++) phi[j] = T2{a.u0, (R)0};
    }
  }
  if constexpr (NV == 2) {
    if (KIND == 2 || KIND == 4) {
      const uint64_t src = (uint64_t)a.lam + vs;
#pragma unroll
      for (int j = 0; j < RN; j++) lam[j] = ld(src, j);
    } else {
#pragma unroll
      for (int j = 0; j < RN; j++) lam[j] = T2{(R)0, (R)0};
    }
  }
  // ---- stage this tile's table entries and the set's LUT in LDS
  if constexpr (need_tab) {
#pragma unroll
    for (uint32_t k = 0; k < kTabChunks; k++) {
      const uint32_t i = t + 256 * k;
      *(uint4 *)(ltab + i * 16 + ((i >> 4) << 4)) = tpre[k];
    }
    if (sp.lut >= 0) {
      const T2 *lsrc = (const T2 *)a.luts + (size_t)sp.lut * a.lut_len;
      for (int i = t; i < a.lut_len; i += 256) llut[i] = lsrc[i];
    }
    if constexpr (SHAPE != 2) {
      const R *vsrc = (const R *)a.vals;
      for (int i = t; i < a.lut_len; i += 256) lval[i] = vsrc[i];
    }
  }

  double acc[NSLOT] = {0.0, 0.0, 0.0};
  double w = sp.w1;
  // ---- part 1: stages H, M, L
  constexpr bool RL1 = KIND == 2 || KIND == 4, XT1 = RL1;
  const uint32_t m1 = a.mask1;
  if constexpr (S1 & 1) stage<R, T, NV, AH, RL1, XT1>(phi, lam, m1, sp.tau1, w, acc[SL_A]);
  if constexpr (S1 & 2) {
    xchgp<R, T, NV, AH, AM, HALF>(lds, phi, lam, t);
    stage<R, T, NV, AM, RL1, XT1>(phi, lam, m1, sp.tau1, w, acc[SL_A]);
  }
  if constexpr (S1 & 4) {
    xchgp<R, T, NV, (S1 & 2) ? AM : AH, AL, HALF>(lds, phi, lam, t);
    stage<R, T, NV, AL, RL1, XT1>(phi, lam, m1, sp.tau1, w, acc[SL_A]);
  }
  constexpr int CM = after_stages<S1, true, AH>();
  // ---- middle: elementwise steps
  // elementwise steps, fixed by kind and shape (see launch_pass_f32)
  constexpr uint32_t MID =
      SHAPE == 0 ? 0u
      : SHAPE == 3 ? (KIND == 1 ? (uint32_t)PF_EXPECT : (uint32_t)PF_GGAMMA)
      : (KIND == 1 ? (uint32_t)PF_PHASE
                   : (KIND == 3 ? (uint32_t)(PF_EXPECT | PF_LAMBDA) : (uint32_t)(PF_GGAMMA | PF_PHASE)));
  if constexpr (MID != 0) {
    __syncthreads();
    middle<R, T, NV, TT, CM, MID>(a, sp, phi, lam, ltab, llut, lval, t, w, acc);
  }
  // ---- part 2: stages L, M, H
  w = sp.w2;
  constexpr bool RL2 = KIND != 1, XT2 = KIND != 1;
  const uint32_t m2 = a.mask2;
  if constexpr (S2 & 4) {
    xchgp<R, T, NV, CM, AL, HALF>(lds, phi, lam, t);
    stage<R, T, NV, AL, RL2, XT2>(phi, lam, m2, sp.tau2, w, acc[SL_C]);
  }
  if constexpr (S2 & 2) {
    xchgp<R, T, NV, (S2 & 4) ? AL : CM, AM, HALF>(lds, phi, lam, t);
    stage<R, T, NV, AM, RL2, XT2>(phi, lam, m2, sp.tau2, w, acc[SL_C]);
  }
  if constexpr (S2 & 1) {
    xchgp<R, T, NV, (S2 & 2) ? AM : ((S2 & 4) ? AL : CM), AH, HALF>(lds, phi, lam, t);
    stage<R, T, NV, AH, RL2, XT2>(phi, lam, m2, sp.tau2, w, acc[SL_C]);
  }
  constexpr int CE = after_stages<S2, false, CM>();
  // ---- store (assignment H)
  if constexpr (KIND == 1 || KIND == 2) {
    if (f & PF_STORE_PHI) {
      xchg1p<R, T, CE, AH, HALF>(lds, phi, t);
      const uint64_t dst = (uint64_t)a.phi_out + vs;
#pragma unroll
      for (int j = 0; j < RN; j++) st(dst, j, phi[j]);
    }
  }
  if constexpr (KIND != 1) {
    if (f & PF_STORE_LAM) {
      xchg1p<R, T, CE, AH, HALF>(lds, lam, t);
      const uint64_t dl = (uint64_t)a.lam + vs;
#pragma unroll
      for (int j = 0; j < RN; j++) st(dl, j, lam[j]);
    }
  }
  // ---- workgroup reduction of the partial sums (fixed order: deterministic)
  if (a.slot_off[0] >= 0 || a.slot_off[1] >= 0 || a.slot_off[2] >= 0) {
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
      double v = acc[s];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      acc[s] = v;
    }
    __syncthreads();
    if ((t & 63) == 0) {
#pragma unroll
      for (int s = 0; s < NSLOT; s++) lred[(t >> 6) * NSLOT + s] = acc[s];
    }
    __syncthreads();
    if (t < NSLOT && a.slot_off[t] >= 0) {
      double v = lred[t] + lred[NSLOT + t];
      v += lred[2 * NSLOT + t] + lred[3 * NSLOT + t];
      a.partials[a.slot_off[t] + (int64_t)q * a.nwg + b] = v;
    }
  }
}

// ============================================================== reductions

// out[q][o] = sum over contributions c < cnt[o] and tiles b < nwg of
// partials[((o * maxc + c) * nsets + q) * nwg + b], in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials,
                                                  const int *__restrict__ cnt, int maxc,
                                                  int nsets, int64_t nwg, int nout,
                                                  double *__restrict__ out) {
  __shared__ double red[256];
  const int o = blockIdx.x, q = blockIdx.y;
  double s = 0.0;
  for (int c = 0; c < cnt[o]; c++) {
    const double *src = partials + (((int64_t)o * maxc + c) * nsets + q) * nwg;
    for (int64_t k = threadIdx.x; k < nwg; k += 256) s += src[k];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)q * nout + o] = red[0];
}

// dst[i] = (re + i im) * src[i ^ flip]
template <typename R>
__global__ void k_scale_copy(const typename Cplx<R>::T2 *__restrict__ src,
                             typename Cplx<R>::T2 *__restrict__ dst, uint64_t N, double re,
                             double im, uint64_t flip) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    typename Cplx<R>::T2 v = src[i ^ flip], o;
    o.x = (R)((double)v.x * re - (double)v.y * im);
    o.y = (R)((double)v.x * im + (double)v.y * re);
    dst[i] = o;
  }
}

// ============================================================== whole-state kernel

// Block-wide sum of one double per thread (256 threads, fixed order).
__device__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

struct DC {
  double re, im;
};
__device__ __forceinline__ DC dmul(DC a, DC b) { return DC{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Rotation parameters of e^{-i beta X} in the unnormalised form (see file header): tau and
// the dropped scalar f of the forward rotation; the inverse rotation uses -tau and finv.
template <typename R>
__device__ void rot_params(double beta, R &tau, DC &f, DC &finv, bool &flip) {
  double sb, cb;
  sincos(beta, &sb, &cb);
  flip = !(fabs(sb) <= fabs(cb));
  if (!flip) {
    tau = (R)(sb / cb);
    double t = (double)tau, nrm = 1.0 / sqrt(1.0 + t * t);
    f = DC{nrm * (cb < 0 ? -1.0 : 1.0), 0.0};
    finv = f;
  } else {
    tau = (R)(-cb / sb);
    double t = (double)tau, s = (sb < 0 ? -1.0 : 1.0) / sqrt(1.0 + t * t);
    f = DC{0.0, -s};
    finv = DC{0.0, s};
  }
}

// One workgroup per (problem, angle set): both vectors and the table in LDS. Forward
// rounds of Eq. (1), <C>, and (grad != 0) the reverse sweep for the gradient.
template <typename R>
__global__ __launch_bounds__(256) void k_small(const SmallItem *__restrict__ items,
                                               const double *__restrict__ angles, int p, int grad,
                                               int max_n, int max_tb, int max_lut,
                                               double *__restrict__ out) {
  using T2 = typename Cplx<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  const SmallItem it = items[blockIdx.x];
  const int n = it.n;
  const uint32_t N = 1u << n;
  T2 *phi = (T2 *)smem;
  T2 *lam = phi + (1u << max_n);
  T2 *lut = lam + (1u << max_n);
  unsigned char *tab = (unsigned char *)(lut + max_lut);
  double *red = (double *)(tab + ((((size_t)max_tb << max_n) + 15) & ~(size_t)15));
  const int tid = threadIdx.x;
  const double *ang = angles + (size_t)it.angle_set * 2 * p;

  for (uint32_t x = tid; x < N; x += 256) {
    if (it.tbytes == 1) ((unsigned char *)tab)[x] = ((const unsigned char *)it.table)[x];
    else ((uint16_t *)tab)[x] = ((const uint16_t *)it.table)[x];
  }
  // the stored vector is the state with the bits of F flipped (tangent form, see the file
  // header): its amplitude at x belongs to basis state x ^ F. F is all bits or none at every
  // phase point; a table with C(~x) = C(x) may ignore it.
  uint32_t F = 0;
  const uint32_t FALL = it.sym ? 0u : N - 1;
  auto cval = [&](uint32_t x) -> uint32_t {
    x ^= F;
    return it.tbytes == 1 ? (uint32_t)tab[x] : (uint32_t)((const uint16_t *)tab)[x];
  };
  auto cost = [&](uint32_t x) -> double { return it.vals[cval(x)]; };
  const R u0 = (R)(1.0 / sqrt((double)N));
  for (uint32_t x = tid; x < N; x += 256) phi[x] = T2{u0, (R)0};
  DC sig{1.0, 0.0};
  auto build_lut = [&](double gamma, double sign) {
    __syncthreads();
    for (int c = tid; c < it.lut_len; c += 256) {
      double s, co;
      sincos(sign * gamma * it.vals[c], &s, &co);
      lut[c] = T2{(R)(sig.re * co - sig.im * s), (R)(sig.re * s + sig.im * co)};
    }
    __syncthreads();
  };
  auto rotate_all = [&](T2 *v, R tau) {
    for (int qb = 0; qb < n; qb++) {
      const uint32_t bit = 1u << qb;
      __syncthreads();
      for (uint32_t i = tid; i < N / 2; i += 256) {
        uint32_t x0 = ((i >> qb) << (qb + 1)) | (i & (bit - 1));
        T2 va = v[x0], vb = v[x0 | bit];
        bfly(va, vb, tau);
        v[x0] = va;
        v[x0 | bit] = vb;
      }
    }
    __syncthreads();
  };

  for (int k = 0; k < p; k++) {
    build_lut(ang[p + k], -1.0);
    for (uint32_t x = tid; x < N; x += 256) {
      T2 L = lut[cval(x)], v = phi[x];
      phi[x] = T2{fmaR(v.x, L.x, -v.y * L.y), fmaR(v.x, L.y, v.y * L.x)};
    }
    sig = DC{1.0, 0.0};
    R tau; DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    rotate_all(phi, tau);
    if (fl) F ^= FALL;
    for (int qb = 0; qb < n; qb++) sig = dmul(sig, f);
  }
  double e = 0.0, nr = 0.0;
  for (uint32_t x = tid; x < N; x += 256) {
    double pr = (double)phi[x].x * phi[x].x + (double)phi[x].y * phi[x].y;
    e += pr * cost(x);
    nr += pr;
  }
  e = block_sum(e, red);
  nr = block_sum(nr, red);
  const double ntrue = (sig.re * sig.re + sig.im * sig.im) * nr;
  double *o = out + (size_t)it.out_index * (1 + 2 * p);
  if (tid == 0) o[0] = e / nr;
  if (!grad) return;

  for (uint32_t x = tid; x < N; x += 256) {
    R kf = (R)(cost(x) - it.c0);
    lam[x] = T2{kf * phi[x].x, kf * phi[x].y};
  }
  __syncthreads();
  for (int k = p - 1; k >= 0; k--) {
    // d/dbeta_k: 2 Im <lam| sum_q X_q |phi>, one term per amplitude pair and qubit
    double gb = 0.0;
    for (int qb = 0; qb < n; qb++) {
      const uint32_t bit = 1u << qb;
      R s = 0;
      for (uint32_t i = tid; i < N / 2; i += 256) {
        uint32_t x0 = ((i >> qb) << (qb + 1)) | (i & (bit - 1));
        s = xpair(phi[x0], phi[x0 | bit], lam[x0], lam[x0 | bit], s);
      }
      gb += (double)s;
    }
    gb = block_sum(gb, red);
    const double wgt = sig.re * sig.re + sig.im * sig.im;
    if (tid == 0) o[1 + k] = 2.0 * wgt * gb / ntrue;
    R tau; DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    rotate_all(phi, -tau);
    rotate_all(lam, -tau);
    if (fl) F ^= FALL;
    for (int qb = 0; qb < n; qb++) sig = dmul(sig, finv);
    // d/dgamma_k: 2 Im <lam| C |phi> = 2 Im <lam| C - c0 |phi> (<lam|phi> is real)
    double gg = 0.0;
    for (uint32_t x = tid; x < N; x += 256) {
      T2 l = lam[x], v = phi[x];
      gg += (double)(fmaR(l.x, v.y, -l.y * v.x)) * (cost(x) - it.c0);
    }
    gg = block_sum(gg, red);
    const double wg2 = sig.re * sig.re + sig.im * sig.im;
    if (tid == 0) o[1 + p + k] = 2.0 * wg2 * gg / ntrue;
    if (k > 0) {
      build_lut(ang[p + k], 1.0);
      for (uint32_t x = tid; x < N; x += 256) {
        T2 L = lut[cval(x)], v = phi[x], l = lam[x];
        phi[x] = T2{fmaR(v.x, L.x, -v.y * L.y), fmaR(v.x, L.y, v.y * L.x)};
        lam[x] = T2{fmaR(l.x, L.x, -l.y * L.y), fmaR(l.x, L.y, l.y * L.x)};
      }
      sig = DC{1.0, 0.0};
      __syncthreads();
    }
  }
}

// ============================================================== whole state in registers

// The same evaluation as k_small for a state of exactly 2^T amplitudes (T = 12, 13), held in
// registers as one tile (TileCfg<T>: 256 threads, 2^(T-8) amplitudes each): a layer is the
// phase multiply in the current register assignment and three register stages joined by two
// LDS exchanges, instead of one LDS pass per qubit. Layers alternate the stage order (H, M, L
// then L, M, H) so the next layer starts in the assignment the last one ended in; the reverse
// sweep undoes each layer in the opposite order, taking the X-pair terms of each group of
// bits before rotating it (weighted by the rotations of the layer done so far, as in the tile
// passes). Scalars, flips and the FP64 sums as in k_small.

// cost-table index of tile element e (the stored vector is flipped by F)
template <typename TT>
__device__ __forceinline__ uint32_t widx(const unsigned char *tab, uint32_t e, uint32_t F) {
  return (uint32_t)((const TT *)tab)[e ^ F];
}

template <typename R, int T, typename TT, int A, int NV>
__device__ __forceinline__ void w_phase(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                        const unsigned char *tab, const typename Cplx<R>::T2 *lut,
                                        uint32_t F, uint32_t t) {
  using T2 = typename Cplx<R>::T2;
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) {
    const T2 L = lut[widx<TT>(tab, elem<A, T>(t, j), F)];
    phi[j] = cmul<T2, R>(phi[j], L);
    if constexpr (NV == 2) lam[j] = cmul<T2, R>(lam[j], L);
  }
}

// <C> and norm partial sums, then lam = (C - c0) phi
template <typename R, int T, typename TT, int A>
__device__ __forceinline__ void w_end(const typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                      const unsigned char *tab, const double *dval, double c0, uint32_t F,
                                      uint32_t t, double &e, double &nr) {
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) {
    const double c = dval[widx<TT>(tab, elem<A, T>(t, j), F)];
    const double pr = (double)phi[j].x * phi[j].x + (double)phi[j].y * phi[j].y;
    e += pr * c;
    nr += pr;
    const R kf = (R)(c - c0);
    lam[j].x = kf * phi[j].x;
    lam[j].y = kf * phi[j].y;
  }
}

// sum of Im(conj(lam) phi) (C - c0)
template <typename R, int T, typename TT, int A>
__device__ __forceinline__ double w_ggamma(const typename Cplx<R>::T2 *phi, const typename Cplx<R>::T2 *lam,
                                           const unsigned char *tab, const double *dval, double c0, uint32_t F,
                                           uint32_t t) {
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) {
    const double c = dval[widx<TT>(tab, elem<A, T>(t, j), F)] - c0;
    g += (double)fmaR(lam[j].x, phi[j].y, -lam[j].y * phi[j].x) * c;
  }
  return g;
}

// Forward mixer of one layer: stages A0, M, A2 (A0 = H, A2 = L when DOWN).
template <typename R, int T, bool DOWN>
__device__ __forceinline__ void w_fwd_mixer(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lds, uint32_t t,
                                            R tau) {
  constexpr int A0 = DOWN ? AH : AL, A2 = DOWN ? AL : AH;
  constexpr uint32_t all = (1u << T) - 1;
  double w = 1.0, acc = 0.0;
  stage<R, T, 1, A0, false, false>(phi, phi, all, tau, w, acc);
  xchg1<R, T, A0, AM>(lds, phi, t);
  stage<R, T, 1, AM, false, false>(phi, phi, all, tau, w, acc);
  xchg1<R, T, AM, A2>(lds, phi, t);
  stage<R, T, 1, A2, false, false>(phi, phi, all, tau, w, acc);
}

// Reverse of a layer whose forward order was DOWN: undo stages A2, M, A0 on both vectors,
// X-pair terms first in each; returns the thread's weighted X-pair sum.
template <typename R, int T, bool DOWN>
__device__ __forceinline__ double w_rev_mixer(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                              typename Cplx<R>::T2 *lds, uint32_t t, R tau) {
  constexpr int A0 = DOWN ? AH : AL, A2 = DOWN ? AL : AH;
  constexpr uint32_t all = (1u << T) - 1;
  double w = 1.0, acc = 0.0;
  stage<R, T, 2, A2, true, true>(phi, lam, all, -tau, w, acc);
  xchg<R, T, 2, A2, AM>(lds, phi, lam, t);
  stage<R, T, 2, AM, true, true>(phi, lam, all, -tau, w, acc);
  xchg<R, T, 2, AM, A0>(lds, phi, lam, t);
  stage<R, T, 2, A0, true, true>(phi, lam, all, -tau, w, acc);
  return acc;
}

template <typename R, int T, typename TT>
__global__ __launch_bounds__(256) void k_whole(const SmallItem *__restrict__ items, const double *__restrict__ angles,
                                               int p, int grad, int max_lut, int pre, double *__restrict__ out) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  constexpr int RN = G::RN;
  constexpr uint32_t N = 1u << T;
  constexpr uint32_t kSlots = N + (N >> Pad<R>::PS);
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *lds = (T2 *)smem;
  T2 *lut = lds + kSlots;
  double *dval = (double *)(lut + max_lut);
  unsigned char *tab = (unsigned char *)(dval + max_lut);
  double *red = (double *)(tab + ((N * sizeof(TT) + 15) & ~15u));
  // pre != 0: every layer's phase table computed once (forward tables, then reverse ones),
  // per-layer scalars, and the per-wave partial gradient sums, reduced after the sweep
  T2 *plut = (T2 *)(red + 4);
  double *scal = (double *)(plut + (size_t)(pre ? 2 * p * max_lut : 0));  // 6 per layer
  double *gsum = scal + (pre ? 6 * p : 0);                                // 8 per layer
  const SmallItem it = items[blockIdx.x];
  const uint32_t t = threadIdx.x;
  const double *ang = angles + (size_t)it.angle_set * 2 * p;

  for (uint32_t i = t; i < N * sizeof(TT) / 4; i += 256) ((uint32_t *)tab)[i] = ((const uint32_t *)it.table)[i];
  for (int c = t; c < it.lut_len; c += 256) dval[c] = it.vals[c];
  uint32_t F = 0;
  const uint32_t FALL = it.sym ? 0u : N - 1;
  DC sig{1.0, 0.0};
  auto lut_entry = [&](const DC &sc, double gamma, double sign, int c) -> T2 {
    double sn, co;
    sincos(sign * gamma * dval[c], &sn, &co);
    return T2{(R)(sc.re * co - sc.im * sn), (R)(sc.re * sn + sc.im * co)};
  };
  auto build_lut = [&](double gamma, double sign) {
    __syncthreads();
    for (int c = t; c < it.lut_len; c += 256) lut[c] = lut_entry(sig, gamma, sign, c);
    __syncthreads();
  };
  if (pre) {
    __syncthreads();  // dval staged
    // scalars of layer k, in the order the sweeps accumulate them: forward table scale
    // (f_{k-1}^T, 1 for k = 0), reverse table scale and weights before and after undoing
    // layer k (the last layer starts from the forward's final scalar)
    for (int k = t; k < p; k += 256) {
      R tau;
      DC f, finv, sf{1.0, 0.0}, before{1.0, 0.0};
      bool fl;
      if (k > 0) {
        rot_params<R>(ang[k - 1], tau, f, finv, fl);
        for (int qb = 0; qb < T; qb++) sf = dmul(sf, f);
      }
      rot_params<R>(ang[k], tau, f, finv, fl);
      if (k == p - 1)
        for (int qb = 0; qb < T; qb++) before = dmul(before, f);
      DC after = before;
      for (int qb = 0; qb < T; qb++) after = dmul(after, finv);
      double *sk = scal + 6 * k;
      sk[0] = sf.re;
      sk[1] = sf.im;
      sk[2] = after.re;
      sk[3] = after.im;
      sk[4] = before.re * before.re + before.im * before.im;
      sk[5] = after.re * after.re + after.im * after.im;
    }
    __syncthreads();
    for (int i = t; i < 2 * p * it.lut_len; i += 256) {
      const int kk = i / it.lut_len, c = i - kk * it.lut_len;
      const bool rev = kk >= p;
      const int k = rev ? kk - p : kk;
      const double *sk = scal + 6 * k;
      const DC sc = rev ? DC{sk[2], sk[3]} : DC{sk[0], sk[1]};
      plut[(size_t)kk * max_lut + c] = lut_entry(sc, ang[p + k], rev ? 1.0 : -1.0, c);
    }
    __syncthreads();
  }

  T2 phi[RN], lam[RN];
  const R u0 = (R)(1.0 / sqrt((double)N));
#pragma unroll
  for (int j = 0; j < RN; j++) phi[j] = T2{u0, (R)0};

  // ---- forward: layer k starts in H when k is even (H, M, L) and in L when odd (L, M, H)
  auto fwd_layer = [&](int k, auto down) {
    constexpr bool D = decltype(down)::value;
    const T2 *lk = lut;
    if (pre) lk = plut + (size_t)k * max_lut;
    else build_lut(ang[p + k], -1.0);
    w_phase<R, T, TT, D ? AH : AL, 1>(phi, lam, tab, lk, F, t);
    sig = DC{1.0, 0.0};
    R tau;
    DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    w_fwd_mixer<R, T, D>(phi, lds, t, tau);
    if (fl) F ^= FALL;
    for (int qb = 0; qb < T; qb++) sig = dmul(sig, f);
  };
  for (int k = 0; k < p; k += 2) {
    fwd_layer(k, std::true_type{});
    if (k + 1 < p) fwd_layer(k + 1, std::false_type{});
  }
  // ends in L after an odd number of layers, in H after an even number
  double e = 0.0, nr = 0.0;
  if (p & 1) w_end<R, T, TT, AL>(phi, lam, tab, dval, it.c0, F, t, e, nr);
  else w_end<R, T, TT, AH>(phi, lam, tab, dval, it.c0, F, t, e, nr);
  e = block_sum(e, red);
  nr = block_sum(nr, red);
  const double ntrue = (sig.re * sig.re + sig.im * sig.im) * nr;
  double *o = out + (size_t)it.out_index * (1 + 2 * p);
  if (t == 0) o[0] = e / nr;
  if (!grad) return;

  // wave sums (the first half of block_sum); with pre they are kept per layer and wave
  auto wave_sum = [&](double v) -> double {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
  };
  // ---- reverse: layer k was DOWN when k is even; undoing it ends in its first assignment
  auto rev_layer = [&](int k, auto down) {
    constexpr bool D = decltype(down)::value;
    constexpr int A0 = D ? AH : AL;
    const double wgt = sig.re * sig.re + sig.im * sig.im;
    R tau;
    DC f, finv;
    bool fl;
    rot_params<R>(ang[k], tau, f, finv, fl);
    const double xb = w_rev_mixer<R, T, D>(phi, lam, lds, t, tau);
    if (pre) {
      const double v = wave_sum(xb);
      if ((t & 63) == 0) gsum[8 * k + (t >> 6)] = v;
    } else {
      const double gb = block_sum(xb, red);
      if (t == 0) o[1 + k] = 2.0 * wgt * gb / ntrue;
    }
    if (fl) F ^= FALL;
    for (int qb = 0; qb < T; qb++) sig = dmul(sig, finv);
    const double xg = w_ggamma<R, T, TT, A0>(phi, lam, tab, dval, it.c0, F, t);
    if (pre) {
      const double v = wave_sum(xg);
      if ((t & 63) == 0) gsum[8 * k + 4 + (t >> 6)] = v;
    } else {
      const double gg = block_sum(xg, red);
      const double wg2 = sig.re * sig.re + sig.im * sig.im;
      if (t == 0) o[1 + p + k] = 2.0 * wg2 * gg / ntrue;
    }
    if (k > 0) {
      const T2 *lk = lut;
      if (pre) lk = plut + (size_t)(p + k) * max_lut;
      else build_lut(ang[p + k], 1.0);
      w_phase<R, T, TT, A0, 2>(phi, lam, tab, lk, F, t);
      sig = DC{1.0, 0.0};
    }
  };
  for (int k = p - 1; k >= 0; k--) {
    if (k & 1) rev_layer(k, std::false_type{});
    else rev_layer(k, std::true_type{});
  }
  if (pre) {  // the block sums, in block_sum's order, and the layer weights
    __syncthreads();
    for (int k = t; k < p; k += 256) {
      const double *gk = gsum + 8 * k, *sk = scal + 6 * k;
      o[1 + k] = 2.0 * sk[4] * ((gk[0] + gk[1]) + (gk[2] + gk[3])) / ntrue;
      o[1 + p + k] = 2.0 * sk[5] * ((gk[4] + gk[5]) + (gk[6] + gk[7])) / ntrue;
    }
  }
}

// ============================================================== Walsh-Hadamard tile pass

// Hadamards on the tile bits in `mask` held in the registers of assignment A.
template <typename R, int T, int A>
__device__ __forceinline__ void hstage(typename Cplx<R>::T2 *v, uint32_t mask) {
  using G = TileCfg<T>;
  const R h = (R)0.70710678118654752440;
#pragma unroll
  for (int b = 0; b < G::RB; b++) {
    constexpr uint32_t grp = group<A, T>();
    const int tb = regbit<A, T>(b);
    if (((grp & mask) >> tb) & 1u) {  // uniform
#pragma unroll
      for (int j = 0; j < G::RN; j++)
        if (!(j & (1 << b))) {
          const typename Cplx<R>::T2 a = v[j], c = v[j | (1 << b)];
          v[j] = typename Cplx<R>::T2{(a.x + c.x) * h, (a.y + c.y) * h};
          v[j | (1 << b)] = typename Cplx<R>::T2{(a.x - c.x) * h, (a.y - c.y) * h};
        }
    }
  }
}

// One pass of the Walsh-Hadamard transform over tiles of 2^T amplitudes held in registers
// (T = 13 for complex64, 12 for complex128): tile bits [0, c) are contiguous index bits (rows),
// tile bits [c, T) are the transformed index bits [b0, b0 + T - c) (c = 0 and b0 = 0 for the
// first pass). Stages H, then M and L as far as the transformed bits reach, with LDS
// exchanges between them; loads and stores in assignment H (lanes over the low tile bits).
template <typename R, int T, int NV, bool PRE>
__global__ __launch_bounds__(256) void k_wht(typename Cplx<R>::T2 *__restrict__ phi,
                                             typename Cplx<R>::T2 *__restrict__ lam, uint64_t N, int b0, int c,
                                             XDiag pre, const typename Cplx<R>::T2 *__restrict__ luts, int lut_len) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *lds = (T2 *)smem;
  const uint32_t t = threadIdx.x;
  const uint64_t r = blockIdx.x;
  const int B = T - c, lo_w = b0 - c;
  const uint64_t base = ((r & ((1ull << lo_w) - 1)) << c) | ((r >> lo_w) << (b0 + B));
  const uint32_t cmask = (1u << c) - 1;
  const uint32_t mask = ((1u << T) - 1) & ~cmask;
  auto addr = [&](uint32_t e) -> uint64_t { return base | (e & cmask) | ((uint64_t)(e >> c) << b0); };
  T2 v[G::RN];
  for (int k = 0; k < NV; k++) {
    T2 *vec = (k == 0 ? phi : lam) + (size_t)blockIdx.y * N;
#pragma unroll
    for (int j = 0; j < G::RN; j++) v[j] = vec[addr(elem<AH, T>(t, j))];
    if constexpr (PRE) {  // the diagonal that precedes this transform, applied on load
      const T2 *lut = luts + (size_t)blockIdx.y * (pre.mode == XD_QUBIT ? 1024 : lut_len);
#pragma unroll
      for (int j = 0; j < G::RN; j++) v[j] = cmul<T2, R>(v[j], xdiag_value(pre, lut, addr(elem<AH, T>(t, j)), N));
    }
    hstage<R, T, AH>(v, mask);
    if (mask & group<AM, T>()) {
      xchg1<R, T, AH, AM>(lds, v, t);
      hstage<R, T, AM>(v, mask);
      if (mask & group<AL, T>()) {
        xchg1<R, T, AM, AL>(lds, v, t);
        hstage<R, T, AL>(v, mask);
        xchg1<R, T, AL, AH>(lds, v, t);
      } else {
        xchg1<R, T, AM, AH>(lds, v, t);
      }
    }
#pragma unroll
    for (int j = 0; j < G::RN; j++) vec[addr(elem<AH, T>(t, j))] = v[j];
  }
}

static int wht_tile_bits(int precision) { return precision == 0 ? 13 : 12; }

// Transformed bits of pass k of an n-qubit transform: the first pass takes the low T bits, the
// others T - 5 bits at a time (rows of 2^5 amplitudes), the last one the remaining B bits with
// T - B contiguous row bits.
static void wht_schedule(int n, int T, std::vector<std::pair<int, int>> &out) {
  int b = 0;
  while (b < n) {
    const int B = b == 0 ? T : (n - b < T - 5 ? n - b : T - 5);
    out.emplace_back(b, b == 0 ? 0 : T - B);
    b += B;
  }
}

template <typename R, int T>
static hipError_t wht_t(int nv, void *phi, void *lam, int n, int nsets, hipStream_t s, const XDiag *pre,
                        const void *luts, int lut_len) {
  using T2 = typename Cplx<R>::T2;
  const uint64_t N = 1ull << n;
  const size_t lds = (size_t)((1u << T) + ((1u << T) >> Pad<R>::PS)) * sizeof(T2);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_wht<R, T, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       96 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_wht<R, T, 1, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              96 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  std::vector<std::pair<int, int>> sched;
  wht_schedule(n, T, sched);
  const dim3 g((unsigned)(1ull << (n - T)), nsets);
  const XDiag none{};
  // one vector per launch: the single-vector kernel keeps two waves per SIMD
  for (int k = 0; k < nv; k++)
    for (size_t i = 0; i < sched.size(); i++) {
      T2 *v = (T2 *)(k == 0 ? phi : lam);
      if (i == 0 && k == 0 && pre)
        k_wht<R, T, 1, true><<<g, 256, lds, s>>>(v, nullptr, N, sched[i].first, sched[i].second, *pre,
                                                 (const T2 *)luts, lut_len);
      else
        k_wht<R, T, 1, false><<<g, 256, lds, s>>>(v, nullptr, N, sched[i].first, sched[i].second, none, nullptr, 0);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t launch_wht_tiles(int precision, int nv, void *phi, void *lam, int n, int nsets, hipStream_t s,
                            const XDiag *pre, const void *luts, int lut_len) {
  if (n < wht_tile_bits(precision)) return hipErrorInvalidValue;
  return precision == 0 ? wht_t<float, 13>(nv, phi, lam, n, nsets, s, pre, luts, lut_len)
                        : wht_t<double, 12>(nv, phi, lam, n, nsets, s, pre, luts, lut_len);
}

int wht_tile_passes(int n, int precision) {
  std::vector<std::pair<int, int>> sched;
  wht_schedule(n, wht_tile_bits(precision), sched);
  return (int)sched.size();
}

int wht_min_bits(int precision) { return wht_tile_bits(precision); }

// ============================================================== launch wrappers

static unsigned grid_for(uint64_t N, unsigned threads) {
  uint64_t g = (N + threads - 1) / threads;
  if (g > 65536 * 4) g = 65536 * 4;
  if (g < 1) g = 1;
  return (unsigned)g;
}

hipError_t launch_cost_table_full(int n, int m, const int32_t *du, const int32_t *dv,
                                  const int32_t *dw, void *table, int tbytes, hipStream_t s) {
  unsigned g = grid_for(1ull << n, 256);
  if (tbytes == 1) k_cost_table_full<uint8_t><<<g, 256, 0, s>>>(n, m, du, dv, dw, (uint8_t *)table);
  else k_cost_table_full<uint16_t><<<g, 256, 0, s>>>(n, m, du, dv, dw, (uint16_t *)table);
  return hipGetLastError();
}

hipError_t launch_cost_table_hw(int n, int k, int m, const int32_t *du, const int32_t *dv,
                                const int32_t *dw, const int64_t *dbinom, uint64_t N,
                                void *table, int tbytes, hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (tbytes == 1)
    k_cost_table_hw<uint8_t><<<g, 256, 0, s>>>(n, k, m, du, dv, dw, dbinom, N, (uint8_t *)table);
  else
    k_cost_table_hw<uint16_t><<<g, 256, 0, s>>>(n, k, m, du, dv, dw, dbinom, N, (uint16_t *)table);
  return hipGetLastError();
}

hipError_t launch_table_max(const void *table, int tbytes, uint64_t N, unsigned *dmax,
                            hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (g > 4096) g = 4096;
  if (tbytes == 1) k_table_max<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)table, N, dmax);
  else k_table_max<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)table, N, dmax);
  return hipGetLastError();
}

hipError_t launch_table_relayout(const void *src, void *dst, int tbytes, int n, int T, int c,
                                 int h0, hipStream_t s) {
  unsigned g = grid_for(1ull << n, 256);
  if (tbytes == 1)
    k_table_relayout<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)src, (uint8_t *)dst, n, T, c, h0);
  else
    k_table_relayout<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)src, (uint16_t *)dst, n, T, c, h0);
  return hipGetLastError();
}

hipError_t launch_table_widen(const void *src, int tbytes, int64_t *dst, uint64_t N,
                              hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (tbytes == 1) k_table_widen<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)src, dst, N);
  else k_table_widen<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)src, dst, N);
  return hipGetLastError();
}

hipError_t launch_luts(int precision, const LutJob *jobs, int njobs, int lut_len, const double *vals,
                       void *luts, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (precision == 0) k_luts<float><<<njobs, 256, 0, s>>>(jobs, lut_len, vals, (float2 *)luts);
  else k_luts<double><<<njobs, 256, 0, s>>>(jobs, lut_len, vals, (double2 *)luts);
  return hipGetLastError();
}

hipError_t launch_table_reverse(const void *src, void *dst, int tbytes, uint64_t count, hipStream_t s) {
  unsigned g = grid_for(count, 256);
  if (tbytes == 1) k_table_reverse<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)src, (uint8_t *)dst, count);
  else k_table_reverse<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)src, (uint16_t *)dst, count);
  return hipGetLastError();
}

hipError_t launch_table_values(const void *table, int tbytes, const double *vals, double *dst, uint64_t N,
                               hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (tbytes == 1) k_table_values<uint8_t><<<g, 256, 0, s>>>((const uint8_t *)table, vals, dst, N);
  else k_table_values<uint16_t><<<g, 256, 0, s>>>((const uint16_t *)table, vals, dst, N);
  return hipGetLastError();
}

template <typename R, int T>
static size_t lds_for(int tbytes, int lut_len, bool half = false) {
  const size_t slots = (size_t)1 << (half ? T - 1 : T);
  size_t st = (slots + (slots >> (sizeof(R) == 4 ? 5 : 4))) * 2 * sizeof(R);
  size_t tb = ((size_t)(1u << T) * tbytes);
  tb += (tb >> 8) * 16;
  return st + tb + (size_t)lut_len * 3 * sizeof(R);
}

size_t pass_lds_bytes(int precision, int tbytes, int lut_len) {
  return precision == 0 ? lds_for<float, TILE_BITS_F32>(tbytes, lut_len)
                        : lds_for<double, TILE_BITS_F64>(tbytes, lut_len);
}

template <typename R, int T, int KIND, int S1, int S2, int SHAPE, typename TT>
static hipError_t launch_pass_t(const PassArgs<R> &a, hipStream_t s) {
  size_t lds = lds_for<R, T>((int)sizeof(TT), a.lut_len, pass_half_xchg<KIND, S1, S2>());
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_pass<R, T, KIND, S1, S2, SHAPE, TT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid(a.nwg, a.nsets);
  hipLaunchKernelGGL((k_pass<R, T, KIND, S1, S2, SHAPE, TT>), grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

// Shapes: 0 = part 1 only; 1 = both parts with the kind's middle steps (forward: phase;
// reverse: gamma gradient and inverse phase; fused: <C> and lam); 2 = part 2 only after the
// phase (first forward pass); 3 = part 1 then a reduction (forward: <C>; reverse: gamma
// gradient).
template <typename R, int T, int KIND, typename TT, int SX>
static hipError_t launch_shape(const PassArgs<R> &a, int shape, hipStream_t s) {
  if constexpr (KIND == 3) return launch_pass_t<R, T, KIND, SX, SX, 1, TT>(a, s);
  else {
    if (shape == 0) return launch_pass_t<R, T, KIND, SX, 0, 0, TT>(a, s);
    if (shape == 3) return launch_pass_t<R, T, KIND, SX, 0, 3, TT>(a, s);
    if constexpr (KIND == 1)
      if (shape == 2) return launch_pass_t<R, T, KIND, 0, SX, 2, TT>(a, s);
    return launch_pass_t<R, T, KIND, SX, SX, 1, TT>(a, s);
  }
}

template <typename R, int T, int KIND, typename TT>
static hipError_t launch_sx(const PassArgs<R> &a, int sx, int shape, hipStream_t s) {
  if (sx == 7) return launch_shape<R, T, KIND, TT, 7>(a, shape, s);
  if (sx == 5) return launch_shape<R, T, KIND, TT, 5>(a, shape, s);
  if (sx == 3) return launch_shape<R, T, KIND, TT, 3>(a, shape, s);
  return launch_shape<R, T, KIND, TT, 1>(a, shape, s);
}

template <typename R, int T, typename TT>
static hipError_t launch_kind(const PassArgs<R> &a, int kind, int sx, int shape, hipStream_t s) {
  if (kind == 1) return launch_sx<R, T, 1, TT>(a, sx, shape, s);
  if (kind == 2) return launch_sx<R, T, 2, TT>(a, sx, shape, s);
  if (kind == 4) return launch_sx<R, T, 4, TT>(a, sx, shape, s);
  return launch_sx<R, T, 3, TT>(a, sx, shape, s);
}

hipError_t launch_pass_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes,
                           hipStream_t s) {
  return tbytes == 1 ? launch_kind<float, TILE_BITS_F32, uint8_t>(a, kind, sx, shape, s)
                     : launch_kind<float, TILE_BITS_F32, uint16_t>(a, kind, sx, shape, s);
}

hipError_t launch_pass_f64(const PassArgs<double> &a, int kind, int sx, int shape, int tbytes,
                           hipStream_t s) {
  return tbytes == 1 ? launch_kind<double, TILE_BITS_F64, uint8_t>(a, kind, sx, shape, s)
                     : launch_kind<double, TILE_BITS_F64, uint16_t>(a, kind, sx, shape, s);
}

hipError_t launch_finalize(const double *partials, const int *cnt, int maxc, int nsets,
                           int64_t nwg, int nout, double *out, hipStream_t s) {
  if (nout <= 0 || nsets <= 0) return hipSuccess;
  k_finalize<<<dim3(nout, nsets), 256, 0, s>>>(partials, cnt, maxc, nsets, nwg, nout, out);
  return hipGetLastError();
}

hipError_t launch_small(int precision, const SmallItem *items, int n_items, int max_n,
                        int max_tbytes, int max_lut, const double *angles, int p, int grad,
                        double *out, hipStream_t s) {
  size_t esz = precision == 0 ? 8 : 16;
  size_t lds = (2ull << max_n) * esz + (size_t)max_lut * esz +
               ((((size_t)max_tbytes << max_n) + 15) & ~(size_t)15) + 64;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_small<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_small<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (precision == 0)
    hipLaunchKernelGGL((k_small<float>), dim3(n_items), dim3(256), lds, s, items, angles, p, grad,
                       max_n, max_tbytes, max_lut, out);
  else
    hipLaunchKernelGGL((k_small<double>), dim3(n_items), dim3(256), lds, s, items, angles, p,
                       grad, max_n, max_tbytes, max_lut, out);
  return hipGetLastError();
}

template <typename R, int T, typename TT>
static hipError_t launch_whole_t(const SmallItem *items, int n_items, int max_lut, const double *angles, int p,
                                 int grad, double *out, hipStream_t s) {
  using T2 = typename Cplx<R>::T2;
  constexpr size_t N = size_t(1) << T;
  const size_t base = (N + (N >> Pad<R>::PS)) * sizeof(T2) + (size_t)max_lut * (sizeof(T2) + sizeof(double)) +
                      ((N * sizeof(TT) + 15) & ~size_t(15)) + 4 * sizeof(double);
  // precomputed phase tables and deferred sums when they fit without lowering occupancy:
  // complex64 at n = 12 keeps two workgroups per CU below 80 KB
  const size_t with_pre = base + (size_t)2 * p * max_lut * sizeof(T2) + (size_t)14 * p * sizeof(double);
  const size_t cap = (sizeof(R) == 4 && T == 12) ? 80 * 1024 : 160 * 1024;
  const int pre = grad && with_pre <= cap ? 1 : 0;
  const size_t lds = pre ? with_pre : base + 64;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_whole<R, T, TT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_whole<R, T, TT>), dim3(n_items), dim3(256), lds, s, items, angles, p, grad, max_lut, pre, out);
  return hipGetLastError();
}

bool whole_supported(int precision, int n) { return precision == 0 ? (n == 12 || n == 13) : n == 12; }

hipError_t launch_whole(int precision, int n, int tbytes, const SmallItem *items, int n_items, int max_lut,
                        const double *angles, int p, int grad, double *out, hipStream_t s) {
  if (precision == 0) {
    if (n == 12)
      return tbytes == 1 ? launch_whole_t<float, 12, uint8_t>(items, n_items, max_lut, angles, p, grad, out, s)
                         : launch_whole_t<float, 12, uint16_t>(items, n_items, max_lut, angles, p, grad, out, s);
    if (n == 13)
      return tbytes == 1 ? launch_whole_t<float, 13, uint8_t>(items, n_items, max_lut, angles, p, grad, out, s)
                         : launch_whole_t<float, 13, uint16_t>(items, n_items, max_lut, angles, p, grad, out, s);
  } else if (n == 12) {
    return tbytes == 1 ? launch_whole_t<double, 12, uint8_t>(items, n_items, max_lut, angles, p, grad, out, s)
                       : launch_whole_t<double, 12, uint16_t>(items, n_items, max_lut, angles, p, grad, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_scale_copy(int precision, const void *src, void *dst, uint64_t N, double re,
                             double im, uint64_t flip, hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (precision == 0)
    k_scale_copy<float><<<g, 256, 0, s>>>((const float2 *)src, (float2 *)dst, N, re, im, flip);
  else
    k_scale_copy<double><<<g, 256, 0, s>>>((const double2 *)src, (double2 *)dst, N, re, im, flip);
  return hipGetLastError();
}

}  // namespace qaoa
