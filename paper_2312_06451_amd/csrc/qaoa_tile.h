// Register-tile building blocks of the tile passes (device code, included by the kernel
// sources): the tile layout and its three register assignments, the padded LDS exchanges, the
// register stages (qubit rotations about X, or about Y for the X-product mixers), the elementwise
// steps between the parts of a pass, and the pass kernel itself.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
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
// (a, b) <- (a - tau b, b + tau a): I - i tau Y, real coefficients (X-product mixers: with
// tau = +-1 it is R_y(+-pi/2) up to the scalar 1/cos(pi/4), and R_y(pi/2) Z R_y(pi/2)^dag = X)
template <typename T2, typename R>
__device__ __forceinline__ void bfly_y(T2 &a, T2 &b, R tau) {
  T2 na, nb;
  na.x = fmaR(-tau, b.x, a.x);
  na.y = fmaR(-tau, b.y, a.y);
  nb.x = fmaR(tau, a.x, b.x);
  nb.y = fmaR(tau, a.y, b.y);
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
template <typename R, int T, int NV, int B, bool ROT_LAM, bool Y>
__device__ __forceinline__ void rot_bit(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam, R tau) {
  using G = TileCfg<T>;
  auto bf = [&](typename Cplx<R>::T2 &a, typename Cplx<R>::T2 &b) {
    if constexpr (Y) bfly_y(a, b, tau);
    else bfly(a, b, tau);
  };
#pragma unroll
  for (int j = 0; j < G::RN; j++)
    if (!(j & (1 << B))) bf(phi[j], phi[j | (1 << B)]);
  if constexpr (NV == 2 && ROT_LAM) {
#pragma unroll
    for (int j = 0; j < G::RN; j++)
      if (!(j & (1 << B))) bf(lam[j], lam[j | (1 << B)]);
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

template <typename R, int T, int NV, int A, bool ROT_LAM, int B, bool Y>
__device__ __forceinline__ void rot_bits(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                         uint32_t mask, R tau, double shrink, double &w) {
  using G = TileCfg<T>;
  if constexpr (B < G::RB) {
    constexpr int tb = regbit<A, T>(B);
    if constexpr ((group<A, T>() >> tb) & 1u) {
      const bool on = (mask >> tb) & 1u;  // uniform
      rot_bit<R, T, NV, B, ROT_LAM, Y>(phi, lam, on ? tau : (R)0);
      if (on) w *= shrink;
    }
    rot_bits<R, T, NV, A, ROT_LAM, B + 1, Y>(phi, lam, mask, tau, shrink, w);
  }
}

// One register stage: every register bit of assignment A whose tile bit belongs to A's group
// is processed; bits in `mask` are rotated (their X-pair terms taken first when XT), the
// others pass. Y: Y rotations (X-product mixers) instead of X rotations.
template <typename R, int T, int NV, int A, bool ROT_LAM, bool XT, bool Y = false>
__device__ __forceinline__ void stage(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                      uint32_t mask, R tau, double &w, double &acc) {
  if constexpr (NV == 2 && XT) {
    xterms<R, T, A, 0>(phi, lam, mask, w, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
  const double shrink = 1.0 / (1.0 + (double)tau * (double)tau);
  rot_bits<R, T, NV, A, ROT_LAM, 0, Y>(phi, lam, mask, tau, shrink, w);
}

// Staged table entry of register j (assignment A) of the thread whose base is tb.
template <typename TT, int T, int A>
__device__ __forceinline__ uint32_t tab_at(const unsigned char *tb, int j) {
  return (uint32_t)(*(const TT *)(tb + toffc<T, A, (int)sizeof(TT)>(j)));
}

// Value index of register j in assignment A for the elementwise steps: the tile's staged table
// entry, or (X-product passes, mixer diagonal by Hamming weight) the popcount of the state index
// y. The thread's and the register's parts of y occupy disjoint bits, so the popcount is the
// sum of the thread part's and the register part's (a constant).
template <typename TT, int T, int A>
struct TabIdx {
  const unsigned char *tb;
  __device__ __forceinline__ uint32_t operator()(int j) const { return tab_at<TT, T, A>(tb, j); }
};
template <int T, int A>
struct PopIdx {
  uint32_t i0;  // popcount of the thread's part of y
  __device__ __forceinline__ uint32_t operator()(int j) const {
    return i0 + (uint32_t)__builtin_popcount(elem<A, T>(0u, (uint32_t)j));
  }
};

// Parity-mask index: the thread part's index XOR register j's (a per-pass constant table).
template <typename P>
struct TermsIdx {
  uint32_t i0;
  const P *a;
  __device__ __forceinline__ uint32_t operator()(int j) const { return i0 ^ (uint32_t)a->xreg[j]; }
};

template <typename T2, typename R>
__device__ __forceinline__ T2 cmul(const T2 &v, const T2 &L) {
  T2 o;
  o.x = fmaR(v.x, L.x, -v.y * L.y);
  o.y = fmaR(v.x, L.y, v.y * L.x);
  return o;
}

// Middle of a per-qubit multi-angle pass (the mixer diagonal e^{-i sum_q beta_q (-1)^{y_q}} in
// the basis of V): the diagonal of state y = y0 | (register j's part) is F(y0) L[j], F(y0) the
// set's constant factor times e^{2i beta_q} over the bits q of y0 (FP64 product, once per
// thread), L[j] the register part's factor from the staged LUT. With GS, first the weighted
// sums of Im(conj(lam) phi): over all of the thread's states (mt) and over those with register
// bit b set (mu[b]); per-thread sums of the 2^RB terms in FP32, then FP64.
template <typename R, int T, int NV, bool GS>
__device__ __forceinline__ void middle_ma(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                          const typename Cplx<R>::T2 *llut, const double2 *bf, uint64_t y0,
                                          double w, double &mt, double *mu) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  if constexpr (NV == 2 && GS) {
    R st = 0, su[G::RB];
#pragma unroll
    for (int b = 0; b < G::RB; b++) su[b] = 0;
#pragma unroll
    for (int j = 0; j < G::RN; j++) {
      const R im = fmaR(lam[j].x, phi[j].y, -lam[j].y * phi[j].x);
      st += im;
#pragma unroll
      for (int b = 0; b < G::RB; b++)
        if (j & (1 << b)) su[b] += im;
    }
    pin(st);
    mt = w * (double)st;
#pragma unroll
    for (int b = 0; b < G::RB; b++) {
      pin(su[b]);
      mu[b] = w * (double)su[b];
    }
  }
  double fr = bf[0].x, fi = bf[0].y;
  for (uint64_t yy = y0; yy; yy &= yy - 1) {
    const double2 f = bf[1 + __builtin_ctzll(yy)];
    const double nr = fr * f.x - fi * f.y;
    fi = fr * f.y + fi * f.x;
    fr = nr;
  }
  const T2 F{(R)fr, (R)fi};
#pragma unroll
  for (int j = 0; j < G::RN; j++) {
    const T2 D = cmul<T2, R>(F, llut[j]);
    phi[j] = cmul<T2, R>(phi[j], D);
    if constexpr (NV == 2) lam[j] = cmul<T2, R>(lam[j], D);
  }
}

// Elementwise steps in assignment A, each step in its own loop (no per-element branching).
// MID != 0 fixes the steps at compile time (flag bits of the PF_ set); MID == 0 reads them
// from the pass flags.
template <typename R, int T, int NV, int A, uint32_t MID, typename IX>
__device__ __forceinline__ void middle(const PassArgs<R> &a, const SetParams<R> &sp,
                                       typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                       const typename Cplx<R>::T2 *llut, const R *lval, const IX &ix,
                                       double w, double *acc) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  constexpr uint32_t f = MID;
  if (f & PF_EXPECT) {
    R e_acc = 0, n_acc = 0;
#pragma unroll
    for (int j = 0; j < G::RN; j++) {
      const R cr = lval[ix(j)];
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
        const R cr = lval[ix(j)];
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
        const R cr = lval[ix(j)] - a.lam_c0;
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
      const T2 L = llut[ix(j)];
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
// S1 / S2: register stages of part 1 / part 2. OP 0: the stages rotate qubits about X
// (transverse-field mixer); OP 1 and 2: about Y, which with tau = +-1 applies the basis change
// of the X-product mixers (Eq. (2) with R_y(pi/2) in place of the Hadamard: both map Z to X),
// with no X-pair terms; OP 1 indexes the middle's diagonal by the cost table, OP 2 by the
// Hamming weight of the state index, OP 3 by its parities against a set of masks, OP 4 is the
// per-qubit multi-angle diagonal (OP 2 to 4: the mixer's diagonal; no table is read).
template <typename R, int T, int KIND, int S1, int S2, int SHAPE, typename TT, int OP = 0, int LAY = 0>
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
  // the state streams through once per pass: non-temporal loads and stores
  auto ld = [&](uint64_t vb, int j) -> T2 { V2 v = __builtin_nontemporal_load(at(vb, j)); return T2{v.x, v.y}; };
  // stores recompute the per-register offsets (from fresh copies of the geometry) instead of
  // keeping the loads' 32 64-bit offsets live across the whole pass
  auto st = [&](uint64_t vb, int j, const T2 &x) {
    const uint32_t cs = fresh_s((uint32_t)a.c), hs = fresh_s((uint32_t)a.h0);
    const uint64_t e = (uint64_t)j << G::TB;
    const uint64_t jb = ((e & ((1ull << cs) - 1)) | ((e >> cs) << hs)) * sizeof(T2);
    V2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, (gV2 *)((gbyte *)uniform64(vb + jb) + tbyte));
  };
  const uint64_t vs = ((uint64_t)q * a.vstride + base) * sizeof(T2);
  // LAY 1..3: the swizzled layout, element x at x ^ (((x >> a.swz_src) & 1023) << a.swz).
  // A tile whose strided bits are the top ones has 2^10 rows a large power of two apart, which
  // in the natural layout share their low address bits and so their L2 channel and DRAM bank;
  // folding the top bits into middle ones spreads them. The map is linear over XOR, so element
  // base | off(t) | off(j) sits at sw(base) ^ sw(off(t)) ^ sw(off(j)): a uniform part (scalar
  // base) and a per-thread part below 2^32 bytes, combined with one XOR per access (LAY 1:
  // non-temporal accesses, LAY 2: cached ones).
  const uint64_t vq = (uint64_t)q * a.vstride * sizeof(T2);
  auto swzf = [](uint64_t x, uint32_t sh, uint32_t src) -> uint64_t { return x ^ (((x >> src) & 1023ull) << sh); };
  auto tswf = [&]() -> uint32_t { return (uint32_t)(swzf(off(t), a.swz, a.swz_src) * sizeof(T2)); };
  auto atz = [&](uint64_t v0, uint32_t ts, int j) -> gV2 * {
    const uint64_t u = swzf(base | off((uint32_t)j << G::TB), a.swz, a.swz_src) * sizeof(T2);
    return (gV2 *)((gbyte *)uniform64(v0 + (u & ~0xffffffffull)) + ((uint32_t)u ^ ts));
  };
  auto ldz = [&](uint64_t v0, uint32_t ts, int j, auto nt) -> T2 {
    V2 v;
    if constexpr (decltype(nt)::value) v = __builtin_nontemporal_load(atz(v0, ts, j));
    else v = *atz(v0, ts, j);
    return T2{v.x, v.y};
  };
  // stores: offsets recomputed from fresh copies of the geometry, as in st
  auto stz = [&](uint64_t v0, uint32_t ts, int j, const T2 &x, auto nt) {
    const uint32_t cs = fresh_s((uint32_t)a.c), hs = fresh_s((uint32_t)a.h0);
    const uint32_t ss = fresh_s((uint32_t)a.swz), sr = fresh_s((uint32_t)a.swz_src);
    const uint64_t e = (uint64_t)j << G::TB;
    const uint64_t u = swzf(base | (e & ((1ull << cs) - 1)) | ((e >> cs) << hs), ss, sr) * sizeof(T2);
    gV2 *ptr = (gV2 *)((gbyte *)uniform64(v0 + (u & ~0xffffffffull)) + ((uint32_t)u ^ ts));
    V2 v;
    v.x = x.x;
    v.y = x.y;
    if constexpr (decltype(nt)::value) __builtin_nontemporal_store(v, ptr);
    else *ptr = v;
  };
  // LAY 3, add form (non-temporal): when the tile's own address bits all lie below the
  // source bits, the swizzle value K is uniform per workgroup and splits into its part on the
  // thread bits' positions and the rest, so that the address is a uniform part plus a
  // per-thread part, as in the natural layout (no per-access XOR).
  const uint64_t Kw = ((base >> a.swz_src) & 1023ull) << a.swz;
  auto tsaf = [&]() -> uint32_t { return (uint32_t)((off(t) ^ (Kw & off(255u))) * sizeof(T2)); };
  auto lda = [&](uint64_t v0, uint32_t ts, int j) -> T2 {
    const uint64_t u = ((base | off((uint32_t)j << G::TB)) ^ (Kw & ~off(255u))) * sizeof(T2);
    V2 v = __builtin_nontemporal_load((gV2 *)((gbyte *)uniform64(v0 + u) + ts));
    return T2{v.x, v.y};
  };
  auto sta = [&](uint64_t v0, uint32_t ts, int j, const T2 &x) {
    const uint32_t cs = fresh_s((uint32_t)a.c), hs = fresh_s((uint32_t)a.h0);
    const uint32_t ss = fresh_s((uint32_t)a.swz), sr = fresh_s((uint32_t)a.swz_src);
    auto dep = [&](uint64_t e) -> uint64_t { return (e & ((1ull << cs) - 1)) | ((e >> cs) << hs); };
    const uint64_t K = ((base >> sr) & 1023ull) << ss;
    const uint64_t u = ((base | dep((uint64_t)j << G::TB)) ^ (K & ~dep(255u))) * sizeof(T2);
    V2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, (gV2 *)((gbyte *)uniform64(v0 + u) + ts));
  };
  // One access form per instantiation (forms chosen at run time would be merged by the
  // compiler into one load sequence with 64-bit per-lane addresses and no cache hint).

  T2 phi[RN];
  T2 lam[NV == 2 ? RN : 1];

  // ---- this tile's table bytes, loaded into registers ahead of the state so that writing
  // them to LDS later waits only for these loads
  constexpr bool need_tab = SHAPE != 0 && OP < 2;
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
      if constexpr (LAY == 0) {
#pragma unroll
        for (int j = 0; j < RN; j++) phi[j] = ld(src, j);
      } else {
        const uint64_t v0 = (uint64_t)a.phi + vq;
        if constexpr (LAY == 3) {
          const uint32_t ts = tsaf();
#pragma unroll
          for (int j = 0; j < RN; j++) phi[j] = lda(v0, ts, j);
        } else {
          const uint32_t ts = tswf();
#pragma unroll
          for (int j = 0; j < RN; j++) phi[j] = ldz(v0, ts, j, std::integral_constant<bool, LAY == 1>{});
        }
      }
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
      if constexpr (LAY == 0) {
        const uint64_t src = (uint64_t)a.lam + vs;
#pragma unroll
        for (int j = 0; j < RN; j++) lam[j] = ld(src, j);
      } else {
        const uint64_t v0 = (uint64_t)a.lam + vq;
        if constexpr (LAY == 3) {
          const uint32_t ts = tsaf();
#pragma unroll
          for (int j = 0; j < RN; j++) lam[j] = lda(v0, ts, j);
        } else {
          const uint32_t ts = tswf();
#pragma unroll
          for (int j = 0; j < RN; j++) lam[j] = ldz(v0, ts, j, std::integral_constant<bool, LAY == 1>{});
        }
      }
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
  }
  if constexpr (SHAPE != 0) {
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
  auto stage1 = [&](auto asg) {
    constexpr int A = decltype(asg)::value;
    stage<R, T, NV, A, RL1, XT1 && OP == 0, OP != 0>(phi, lam, m1, sp.tau1, w, acc[SL_A]);
  };
  if constexpr (S1 & 1) stage1(std::integral_constant<int, AH>{});
  if constexpr (S1 & 2) {
    xchgp<R, T, NV, AH, AM, HALF>(lds, phi, lam, t);
    stage1(std::integral_constant<int, AM>{});
  }
  if constexpr (S1 & 4) {
    xchgp<R, T, NV, (S1 & 2) ? AM : AH, AL, HALF>(lds, phi, lam, t);
    stage1(std::integral_constant<int, AL>{});
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
    if constexpr (OP == 2) {
      // the mixer's diagonal, indexed by the Hamming weight of the state index
      const uint64_t y0 = base | off(elem<CM, T>(t, 0u));
      middle<R, T, NV, CM, MID>(a, sp, phi, lam, llut, lval, PopIdx<T, CM>{(uint32_t)__popcll(y0)}, w, acc);
    } else if constexpr (OP == 4) {
      // the per-qubit multi-angle diagonal (shape 1, kinds 1 and 4)
      const uint64_t y0 = base | off(elem<CM, T>(t, 0u));
      double ma_t = 0.0, ma_u[G::RB];
      middle_ma<R, T, NV, KIND == 2 || KIND == 4>(phi, lam, llut, (const double2 *)a.vals + (size_t)q * 33, y0, w,
                                                   ma_t, ma_u);
      if constexpr (KIND == 2 || KIND == 4) {
        // per-qubit sums, reduced here (the table area of LDS is free in these passes): the
        // total, the register-bit sums, and the thread-bit sums (thread bit i: the total of
        // the threads with bit i set), one at a time in a fixed order; a qubit on the tile
        // index takes the total or zero
        constexpr int NS = 1 + G::RB + 8;
        double *red = (double *)ltab;
#pragma unroll
        for (int k = 0; k < NS; k++) {
          double v = k == 0 ? ma_t : (k <= G::RB ? ma_u[k - 1] : (((t >> (k - 1 - G::RB)) & 1u) ? ma_t : 0.0));
          for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
          if ((t & 63) == 0) red[(t >> 6) * NS + k] = v;
        }
        __syncthreads();
        if (t <= (uint32_t)a.n) {
          auto tot = [&](int k) { return (red[k] + red[NS + k]) + (red[2 * NS + k] + red[3 * NS + k]); };
          double val;
          int64_t slot;
          if (t == (uint32_t)a.n) {
            val = tot(0);
            slot = a.ma_total;
          } else {
            const int src = a.ma_src[t];
            if (src < 8) val = tot(1 + src);
            else if (src < 16) val = tot(1 + G::RB + (src - 8));
            else val = ((base >> t) & 1ull) ? tot(0) : 0.0;
            slot = a.ma_slot + (int64_t)t * a.ma_stride;
          }
          a.partials[slot + (int64_t)q * a.nwg + b] = val;
        }
      }
    } else if constexpr (OP == 3) {
      // the mixer's diagonal, indexed by the parities of the state index against the masks
      const uint64_t y0 = base | off(elem<CM, T>(t, 0u));
      uint32_t i0 = 0;
#pragma unroll
      for (int k = 0; k < XD_MAX_TERMS; k++)
        if (k < a.xnterms) i0 |= (uint32_t)(__popcll(y0 & a.xmasks[k]) & 1) << k;
      middle<R, T, NV, CM, MID>(a, sp, phi, lam, llut, lval, TermsIdx<PassArgs<R>>{i0, &a}, w, acc);
    } else {
      const TabIdx<TT, T, CM> tix{ltab + tbase<T, CM, (int)sizeof(TT)>(t)};
      middle<R, T, NV, CM, MID>(a, sp, phi, lam, llut, lval, tix, w, acc);
    }
  }
  // ---- part 2: stages L, M, H
  w = sp.w2;
  constexpr bool RL2 = KIND != 1, XT2 = KIND != 1;
  const uint32_t m2 = a.mask2;
  auto stage2 = [&](auto asg) {
    constexpr int A = decltype(asg)::value;
    stage<R, T, NV, A, RL2, XT2 && OP == 0, OP != 0>(phi, lam, m2, sp.tau2, w, acc[SL_C]);
  };
  if constexpr (S2 & 4) {
    xchgp<R, T, NV, CM, AL, HALF>(lds, phi, lam, t);
    stage2(std::integral_constant<int, AL>{});
  }
  if constexpr (S2 & 2) {
    xchgp<R, T, NV, (S2 & 4) ? AL : CM, AM, HALF>(lds, phi, lam, t);
    stage2(std::integral_constant<int, AM>{});
  }
  if constexpr (S2 & 1) {
    xchgp<R, T, NV, (S2 & 2) ? AM : ((S2 & 4) ? AL : CM), AH, HALF>(lds, phi, lam, t);
    stage2(std::integral_constant<int, AH>{});
  }
  constexpr int CE = after_stages<S2, false, CM>();
  // ---- store (assignment H)
  if constexpr (KIND == 1 || KIND == 2) {
    if (f & PF_STORE_PHI) {
      xchg1p<R, T, CE, AH, HALF>(lds, phi, t);
      if constexpr (LAY == 0) {
        const uint64_t dst = (uint64_t)a.phi_out + vs;
#pragma unroll
        for (int j = 0; j < RN; j++) st(dst, j, phi[j]);
      } else {
        const uint64_t v0 = (uint64_t)a.phi_out + vq;
        if constexpr (LAY == 3) {
          const uint32_t ts = tsaf();
#pragma unroll
          for (int j = 0; j < RN; j++) sta(v0, ts, j, phi[j]);
        } else {
          const uint32_t ts = tswf();
#pragma unroll
          for (int j = 0; j < RN; j++) stz(v0, ts, j, phi[j], std::integral_constant<bool, LAY == 1>{});
        }
      }
    }
  }
  if constexpr (KIND != 1) {
    if (f & PF_STORE_LAM) {
      xchg1p<R, T, CE, AH, HALF>(lds, lam, t);
      if constexpr (LAY == 0) {
        const uint64_t dl = (uint64_t)a.lam + vs;
#pragma unroll
        for (int j = 0; j < RN; j++) st(dl, j, lam[j]);
      } else {
        const uint64_t v0 = (uint64_t)a.lam + vq;
        if constexpr (LAY == 3) {
          const uint32_t ts = tsaf();
#pragma unroll
          for (int j = 0; j < RN; j++) sta(v0, ts, j, lam[j]);
        } else {
          const uint32_t ts = tswf();
#pragma unroll
          for (int j = 0; j < RN; j++) stz(v0, ts, j, lam[j], std::integral_constant<bool, LAY == 1>{});
        }
      }
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

// ---- host side: LDS size and launch of one pass instantiation

template <typename R, int T>
static size_t lds_for(int tbytes, int lut_len, bool half = false) {
  const size_t slots = (size_t)1 << (half ? T - 1 : T);
  size_t st = (slots + (slots >> (sizeof(R) == 4 ? 5 : 4))) * 2 * sizeof(R);
  size_t tb = ((size_t)(1u << T) * tbytes);
  tb += (tb >> 8) * 16;
  return st + tb + (size_t)lut_len * 3 * sizeof(R);
}

template <typename R, int T, int KIND, int S1, int S2, int SHAPE, typename TT, int OP = 0, int LAY = 0>
static hipError_t launch_pass_t(const PassArgs<R> &a, hipStream_t s) {
  size_t lds = lds_for<R, T>((int)sizeof(TT), a.lut_len, pass_half_xchg<KIND, S1, S2>());
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_pass<R, T, KIND, S1, S2, SHAPE, TT, OP, LAY>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid(a.nwg, a.nsets);
  hipLaunchKernelGGL((k_pass<R, T, KIND, S1, S2, SHAPE, TT, OP, LAY>), grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

// Shapes: 0 = part 1 only; 1 = both parts with the kind's middle steps (forward: phase;
// reverse: gamma gradient and inverse phase; fused: <C> and lam); 2 = part 2 only after the
// phase (first forward pass); 3 = part 1 then a reduction (forward: <C>; reverse: gamma
// gradient).
template <typename R, int T, int KIND, typename TT, int SX, int LAY>
static hipError_t launch_shape(const PassArgs<R> &a, int shape, hipStream_t s) {
  if constexpr (KIND == 3) return launch_pass_t<R, T, KIND, SX, SX, 1, TT, 0, LAY>(a, s);
  else {
    if (shape == 0) return launch_pass_t<R, T, KIND, SX, 0, 0, TT, 0, LAY>(a, s);
    if (shape == 3) return launch_pass_t<R, T, KIND, SX, 0, 3, TT, 0, LAY>(a, s);
    if constexpr (KIND == 1)
      if (shape == 2) return launch_pass_t<R, T, KIND, 0, SX, 2, TT, 0, LAY>(a, s);
    return launch_pass_t<R, T, KIND, SX, SX, 1, TT, 0, LAY>(a, s);
  }
}

}  // namespace qaoa
