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
// G(tau) = I - i tau X (tau = tan b; four FMAs per amplitude pair), or, when |tan b| > 1, as
// X G(tau) with tau = -cot b (the output-swapped form). The dropped factor (cos b, or
// -i sin b) is a scalar per vector that the host tracks and folds into the next phase
// lookup table, so every rotation is exactly unitary up to that scalar and norm drift does
// not accumulate.
//
// Tile passes. A workgroup of 256 threads holds a tile of 2^T amplitudes in registers
// (2^(T-8) per thread and vector). Tile bits [0,c) are contiguous address bits; the other
// T-c tile bits sit on a contiguous range of higher address bits. Rotations on tile bits that
// live in a thread's registers need no communication; three register assignments (H, M, L)
// cover all tile bits and the tile moves between them through a padded, bank-conflict-free
// LDS buffer. The phase multiply, the <C> reduction, the adjoint initialisation and the
// gradient inner products are fused into the passes.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "qaoa_internal.h"

namespace qaoa {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T2 = float2; };
template <> struct Cplx<double> { using T2 = double2; };

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

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

// ============================================================== phase lookup tables

// luts[j][c] = s_j * exp(sign_j * i * gamma_j * c): FP64 argument and sincos, one rounding.
template <typename R>
__global__ void k_luts(const LutJob *__restrict__ jobs, int lut_len,
                       typename Cplx<R>::T2 *__restrict__ luts) {
  const LutJob J = jobs[blockIdx.x];
  for (int c = threadIdx.x; c < lut_len; c += blockDim.x) {
    double s, co;
    sincos(J.sign * J.gamma * (double)c, &s, &co);
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

// Padded LDS slot of tile element e (one pad slot per 256 bytes: conflict-free in H, M, L).
template <typename R>
__device__ __forceinline__ uint32_t lpos(uint32_t e) {
  return e + (e >> (sizeof(R) == 4 ? 5 : 4));
}
// Padded byte position of the staged table entry e (16 pad bytes per 256 entries).
__device__ __forceinline__ uint32_t tpos(uint32_t e) { return e + ((e >> 8) << 4); }

template <typename R, int T, int A>
__device__ __forceinline__ void to_lds(typename Cplx<R>::T2 *lds, const typename Cplx<R>::T2 *v,
                                       uint32_t t) {
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) lds[lpos<R>(elem<A, T>(t, j))] = v[j];
}
template <typename R, int T, int A>
__device__ __forceinline__ void from_lds(const typename Cplx<R>::T2 *lds,
                                         typename Cplx<R>::T2 *v, uint32_t t) {
#pragma unroll
  for (int j = 0; j < TileCfg<T>::RN; j++) v[j] = lds[lpos<R>(elem<A, T>(t, j))];
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

template <typename R, int T, int NV, int TO>
__device__ __forceinline__ void move_to(int &cur, typename Cplx<R>::T2 *lds,
                                        typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                        uint32_t t) {
  if (cur == TO) return;
  if (cur == AH) {
    xchg1<R, T, AH, TO>(lds, phi, t);
    if constexpr (NV == 2) xchg1<R, T, AH, TO>(lds, lam, t);
  } else if (cur == AM) {
    xchg1<R, T, AM, TO>(lds, phi, t);
    if constexpr (NV == 2) xchg1<R, T, AM, TO>(lds, lam, t);
  } else {
    xchg1<R, T, AL, TO>(lds, phi, t);
    if constexpr (NV == 2) xchg1<R, T, AL, TO>(lds, lam, t);
  }
  cur = TO;
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
// (a, b) <- (b - i tau a, a - i tau b): X applied after G(tau)
template <typename T2, typename R>
__device__ __forceinline__ void bfly_swap(T2 &a, T2 &b, R tau) {
  T2 na, nb;
  na.x = fmaR(tau, a.y, b.x);
  na.y = fmaR(-tau, a.x, b.y);
  nb.x = fmaR(tau, b.y, a.x);
  nb.y = fmaR(-tau, b.x, a.y);
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

// One register stage: for every register bit of assignment A whose tile bit is in `mask`
// (and owned by A): optionally accumulate the X-pair terms, then rotate.
template <typename R, int T, int NV, int A>
__device__ __forceinline__ void stage(typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                      uint32_t mask, R tau, int swap, bool rot_lam, bool xt,
                                      double &w, double &acc) {
  using G = TileCfg<T>;
  const double shrink = 1.0 / (1.0 + (double)tau * (double)tau);
#pragma unroll
  for (int b = 0; b < G::RB; b++) {
    constexpr uint32_t grp = group<A, T>();
    const int tb = regbit<A, T>(b);
    if (!((grp >> tb) & 1u)) continue;
    if (!((mask >> tb) & 1u)) continue;
    if constexpr (NV == 2) {
      if (xt) {
        R s = 0;
#pragma unroll
        for (int j = 0; j < G::RN; j++)
          if (!(j & (1 << b))) s = xpair(phi[j], phi[j | (1 << b)], lam[j], lam[j | (1 << b)], s);
        acc += w * (double)s;
      }
    }
    if (swap) {
#pragma unroll
      for (int j = 0; j < G::RN; j++)
        if (!(j & (1 << b))) bfly_swap(phi[j], phi[j | (1 << b)], tau);
      if constexpr (NV == 2) {
        if (rot_lam) {
#pragma unroll
          for (int j = 0; j < G::RN; j++)
            if (!(j & (1 << b))) bfly_swap(lam[j], lam[j | (1 << b)], tau);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < G::RN; j++)
        if (!(j & (1 << b))) bfly(phi[j], phi[j | (1 << b)], tau);
      if constexpr (NV == 2) {
        if (rot_lam) {
#pragma unroll
          for (int j = 0; j < G::RN; j++)
            if (!(j & (1 << b))) bfly(lam[j], lam[j | (1 << b)], tau);
        }
      }
    }
    w *= shrink;
  }
}

template <typename R, int T, int NV, typename TT, int A>
__device__ __forceinline__ void middle(const PassArgs<R> &a, const SetParams<R> &sp,
                                       typename Cplx<R>::T2 *phi, typename Cplx<R>::T2 *lam,
                                       const unsigned char *ltab,
                                       const typename Cplx<R>::T2 *llut, uint32_t t, double w,
                                       double *acc) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  const uint32_t f = a.flags;
  R e_acc = 0, n_acc = 0, g_acc = 0;
#pragma unroll
  for (int j = 0; j < G::RN; j++) {
    const uint32_t e = elem<A, T>(t, j);
    const uint32_t cv = (uint32_t)(*(const TT *)(ltab + tpos(e * sizeof(TT))));
    const R cr = (R)cv;
    if (f & PF_EXPECT) {
      R pr = fmaR(phi[j].x, phi[j].x, phi[j].y * phi[j].y);
      e_acc = fmaR(pr, cr, e_acc);
      n_acc += pr;
    }
    if constexpr (NV == 2) {
      if (f & PF_LAMBDA) {
        R kf = sp.lam_rho * (cr - a.lam_c0);
        lam[j].x = kf * phi[j].x;
        lam[j].y = kf * phi[j].y;
      }
      if (f & PF_GGAMMA) {
        R im = fmaR(lam[j].x, phi[j].y, -lam[j].y * phi[j].x);
        g_acc = fmaR(im, cr, g_acc);
      }
    }
    if (f & PF_PHASE) {
      const T2 L = llut[cv];
      T2 o;
      o.x = fmaR(phi[j].x, L.x, -phi[j].y * L.y);
      o.y = fmaR(phi[j].x, L.y, phi[j].y * L.x);
      phi[j] = o;
      if constexpr (NV == 2) {
        if (f & PF_PHASE_BOTH) {
          o.x = fmaR(lam[j].x, L.x, -lam[j].y * L.y);
          o.y = fmaR(lam[j].x, L.y, lam[j].y * L.x);
          lam[j] = o;
        }
      }
    }
  }
  if (f & PF_EXPECT) {
    acc[SL_A] += (double)e_acc;
    acc[SL_B] += (double)n_acc;
  }
  if (f & PF_GGAMMA) acc[SL_B] += w * (double)g_acc;
}

template <typename R, int T, int NV, typename TT>
__global__ __launch_bounds__(256) void k_pass(const PassArgs<R> a) {
  using G = TileCfg<T>;
  using T2 = typename Cplx<R>::T2;
  constexpr int RN = G::RN;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr uint32_t kStateSlots = (1u << T) + ((1u << T) >> (sizeof(R) == 4 ? 5 : 4));
  constexpr uint32_t kTabBytes = ((1u << T) * sizeof(TT)) + (((1u << T) * sizeof(TT)) >> 8) * 16;
  T2 *lds = (T2 *)smem;
  unsigned char *ltab = smem + kStateSlots * sizeof(T2);
  T2 *llut = (T2 *)(ltab + kTabBytes);
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
  auto off = [&](uint32_t e) -> uint64_t {
    return ((uint64_t)e & cmask) | (((uint64_t)e >> a.c) << a.h0);
  };
  const uint64_t tb = base + off(t);
  const uint64_t vs = (uint64_t)q * a.vstride;

  T2 phi[RN];
  T2 lam[NV == 2 ? RN : 1];

  // ---- load (assignment H: lanes run over contiguous address bits)
  if (f & PF_LOAD_PHI) {
    const T2 *src = (const T2 *)a.phi + vs;
#pragma unroll
    for (int j = 0; j < RN; j++) phi[j] = src[tb + off((uint32_t)j << G::TB)];
  } else if (f & PF_LOAD_PSI0) {
    const T2 *src = (const T2 *)a.psi0;
#pragma unroll
    for (int j = 0; j < RN; j++) phi[j] = src[tb + off((uint32_t)j << G::TB)];
  } else {
#pragma unroll
    for (int j = 0; j < RN; j++) {
      phi[j].x = a.u0;
      phi[j].y = (R)0;
    }
  }
  if constexpr (NV == 2) {
    if (f & PF_LOAD_LAM) {
      const T2 *src = (const T2 *)a.lam + vs;
#pragma unroll
      for (int j = 0; j < RN; j++) lam[j] = src[tb + off((uint32_t)j << G::TB)];
    } else {
#pragma unroll
      for (int j = 0; j < RN; j++) lam[j] = T2{(R)0, (R)0};
    }
  }
  // ---- stage this tile's table entries and the set's LUT in LDS
  const bool need_tab = (f & (PF_EXPECT | PF_LAMBDA | PF_GGAMMA | PF_PHASE)) != 0;
  if (need_tab) {
    constexpr uint32_t nchunk = ((1u << T) * sizeof(TT)) / 16;
    const uint4 *src = (const uint4 *)((const unsigned char *)a.table +
                                       (uint64_t)r * ((1ull << T) * sizeof(TT)));
    for (uint32_t i = t; i < nchunk; i += 256) *(uint4 *)(ltab + tpos(i * 16)) = src[i];
    if ((f & PF_PHASE) && sp.lut >= 0) {
      const T2 *lsrc = (const T2 *)a.luts + (size_t)sp.lut * a.lut_len;
      for (int i = t; i < a.lut_len; i += 256) llut[i] = lsrc[i];
    }
  }

  double acc[NSLOT] = {0.0, 0.0, 0.0};
  double w = sp.w1;
  int cur = AH;
  // ---- part 1: stages H, M, L
  {
    const uint32_t m1 = a.mask1;
    const bool rl = (f & PF_ROT1_BOTH) != 0, xt = (f & PF_XT1) != 0;
    if (m1 & group<AH, T>()) {
      move_to<R, T, NV, AH>(cur, lds, phi, lam, t);
      stage<R, T, NV, AH>(phi, lam, m1, sp.tau1, sp.swap1, rl, xt, w, acc[SL_A]);
    }
    if (m1 & group<AM, T>()) {
      move_to<R, T, NV, AM>(cur, lds, phi, lam, t);
      stage<R, T, NV, AM>(phi, lam, m1, sp.tau1, sp.swap1, rl, xt, w, acc[SL_A]);
    }
    if (m1 & group<AL, T>()) {
      move_to<R, T, NV, AL>(cur, lds, phi, lam, t);
      stage<R, T, NV, AL>(phi, lam, m1, sp.tau1, sp.swap1, rl, xt, w, acc[SL_A]);
    }
  }
  // ---- middle: elementwise steps in the current assignment
  if (need_tab) {
    __syncthreads();
    if (cur == AH) middle<R, T, NV, TT, AH>(a, sp, phi, lam, ltab, llut, t, w, acc);
    else if (cur == AM) middle<R, T, NV, TT, AM>(a, sp, phi, lam, ltab, llut, t, w, acc);
    else middle<R, T, NV, TT, AL>(a, sp, phi, lam, ltab, llut, t, w, acc);
  }
  // ---- part 2: stages L, M, H
  w = sp.w2;
  {
    const uint32_t m2 = a.mask2;
    const bool rl = (f & PF_ROT2_BOTH) != 0, xt = (f & PF_XT2) != 0;
    if (m2 & group<AL, T>()) {
      move_to<R, T, NV, AL>(cur, lds, phi, lam, t);
      stage<R, T, NV, AL>(phi, lam, m2, sp.tau2, sp.swap2, rl, xt, w, acc[SL_C]);
    }
    if (m2 & group<AM, T>()) {
      move_to<R, T, NV, AM>(cur, lds, phi, lam, t);
      stage<R, T, NV, AM>(phi, lam, m2, sp.tau2, sp.swap2, rl, xt, w, acc[SL_C]);
    }
    if (m2 & group<AH, T>()) {
      move_to<R, T, NV, AH>(cur, lds, phi, lam, t);
      stage<R, T, NV, AH>(phi, lam, m2, sp.tau2, sp.swap2, rl, xt, w, acc[SL_C]);
    }
  }
  // ---- store (assignment H)
  if (f & (PF_STORE_PHI | PF_STORE_LAM)) {
    move_to<R, T, NV, AH>(cur, lds, phi, lam, t);
    if (f & PF_STORE_PHI) {
      T2 *dst = (T2 *)a.phi + vs;
      if (f & PF_SCALE_OUT) {
#pragma unroll
        for (int j = 0; j < RN; j++) {
          T2 o;
          o.x = fmaR(phi[j].x, sp.out_re, -phi[j].y * sp.out_im);
          o.y = fmaR(phi[j].x, sp.out_im, phi[j].y * sp.out_re);
          phi[j] = o;
        }
      }
#pragma unroll
      for (int j = 0; j < RN; j++) dst[tb + off((uint32_t)j << G::TB)] = phi[j];
    }
    if constexpr (NV == 2) {
      if (f & PF_STORE_LAM) {
        T2 *dst = (T2 *)a.lam + vs;
#pragma unroll
        for (int j = 0; j < RN; j++) dst[tb + off((uint32_t)j << G::TB)] = lam[j];
      }
    }
  }
  // ---- workgroup reduction of the partial sums (fixed order: deterministic)
  bool any = false;
#pragma unroll
  for (int s = 0; s < NSLOT; s++) any |= a.slot_off[s] >= 0;
  if (any) {
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

template <typename R>
__global__ void k_scale_copy(const typename Cplx<R>::T2 *__restrict__ src,
                             typename Cplx<R>::T2 *__restrict__ dst, uint64_t N, double re,
                             double im) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    typename Cplx<R>::T2 v = src[i], o;
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

// Rotation parameters of e^{-i beta X} in the unnormalised form (see file header):
// tau, swap flag and the dropped scalar factor f (forward); the inverse uses -tau, the same
// swap flag and conj-type factor finv.
template <typename R>
__device__ void rot_params(double beta, R &tau, int &swap, DC &f, DC &finv) {
  double sb, cb;
  sincos(beta, &sb, &cb);
  if (fabs(sb) <= fabs(cb)) {
    tau = (R)(sb / cb);
    swap = 0;
    double t = (double)tau, nrm = 1.0 / sqrt(1.0 + t * t);
    f = DC{nrm * (cb < 0 ? -1.0 : 1.0), 0.0};
    finv = f;
  } else {
    tau = (R)(-cb / sb);
    swap = 1;
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
  auto cval = [&](uint32_t x) -> uint32_t {
    return it.tbytes == 1 ? (uint32_t)tab[x] : (uint32_t)((const uint16_t *)tab)[x];
  };
  const R u0 = (R)(1.0 / sqrt((double)N));
  for (uint32_t x = tid; x < N; x += 256) phi[x] = T2{u0, (R)0};
  DC sig{1.0, 0.0};
  auto build_lut = [&](double gamma, double sign) {
    __syncthreads();
    for (int c = tid; c < it.lut_len; c += 256) {
      double s, co;
      sincos(sign * gamma * (double)c, &s, &co);
      lut[c] = T2{(R)(sig.re * co - sig.im * s), (R)(sig.re * s + sig.im * co)};
    }
    __syncthreads();
  };
  auto rotate_all = [&](T2 *v, R tau, int swap) {
    for (int qb = 0; qb < n; qb++) {
      const uint32_t bit = 1u << qb;
      __syncthreads();
      for (uint32_t i = tid; i < N / 2; i += 256) {
        uint32_t x0 = ((i >> qb) << (qb + 1)) | (i & (bit - 1));
        T2 va = v[x0], vb = v[x0 | bit];
        if (swap) bfly_swap(va, vb, tau); else bfly(va, vb, tau);
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
    R tau; int swap; DC f, finv;
    rot_params<R>(ang[k], tau, swap, f, finv);
    rotate_all(phi, tau, swap);
    for (int qb = 0; qb < n; qb++) sig = dmul(sig, f);
  }
  double e = 0.0, nr = 0.0;
  for (uint32_t x = tid; x < N; x += 256) {
    double pr = (double)phi[x].x * phi[x].x + (double)phi[x].y * phi[x].y;
    e += pr * (double)cval(x);
    nr += pr;
  }
  e = block_sum(e, red);
  nr = block_sum(nr, red);
  const double ntrue = (sig.re * sig.re + sig.im * sig.im) * nr;
  double *o = out + (size_t)it.out_index * (1 + 2 * p);
  if (tid == 0) o[0] = e / nr;
  if (!grad) return;

  for (uint32_t x = tid; x < N; x += 256) {
    R kf = (R)((double)cval(x) - it.c0);
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
    R tau; int swap; DC f, finv;
    rot_params<R>(ang[k], tau, swap, f, finv);
    rotate_all(phi, -tau, swap);
    rotate_all(lam, -tau, swap);
    for (int qb = 0; qb < n; qb++) sig = dmul(sig, finv);
    // d/dgamma_k: 2 Im <lam| C |phi>
    double gg = 0.0;
    for (uint32_t x = tid; x < N; x += 256) {
      T2 l = lam[x], v = phi[x];
      gg += (double)(fmaR(l.x, v.y, -l.y * v.x)) * (double)cval(x);
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

hipError_t launch_luts(int precision, const LutJob *jobs, int njobs, int lut_len, void *luts,
                       hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (precision == 0) k_luts<float><<<njobs, 256, 0, s>>>(jobs, lut_len, (float2 *)luts);
  else k_luts<double><<<njobs, 256, 0, s>>>(jobs, lut_len, (double2 *)luts);
  return hipGetLastError();
}

template <typename R, int T>
static size_t lds_for(int tbytes, int lut_len) {
  size_t st = ((1u << T) + ((1u << T) >> (sizeof(R) == 4 ? 5 : 4))) * 2 * sizeof(R);
  size_t tb = ((size_t)(1u << T) * tbytes);
  tb += (tb >> 8) * 16;
  return st + tb + (size_t)lut_len * 2 * sizeof(R);
}

size_t pass_lds_bytes(int precision, int tbytes, int lut_len) {
  return precision == 0 ? lds_for<float, TILE_BITS_F32>(tbytes, lut_len)
                        : lds_for<double, TILE_BITS_F64>(tbytes, lut_len);
}

template <typename R, int T, int NV, typename TT>
static hipError_t launch_pass_t(const PassArgs<R> &a, hipStream_t s) {
  size_t lds = lds_for<R, T>((int)sizeof(TT), a.lut_len);
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute((const void *)k_pass<R, T, NV, TT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        160 * 1024);
    attr_set = true;
  }
  dim3 grid(a.nwg, a.nsets);
  hipLaunchKernelGGL((k_pass<R, T, NV, TT>), grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_pass_f32(const PassArgs<float> &a, int nv, int tbytes, hipStream_t s) {
  constexpr int T = TILE_BITS_F32;
  if (nv == 1) return tbytes == 1 ? launch_pass_t<float, T, 1, uint8_t>(a, s)
                                  : launch_pass_t<float, T, 1, uint16_t>(a, s);
  return tbytes == 1 ? launch_pass_t<float, T, 2, uint8_t>(a, s)
                     : launch_pass_t<float, T, 2, uint16_t>(a, s);
}

hipError_t launch_pass_f64(const PassArgs<double> &a, int nv, int tbytes, hipStream_t s) {
  constexpr int T = TILE_BITS_F64;
  if (nv == 1) return tbytes == 1 ? launch_pass_t<double, T, 1, uint8_t>(a, s)
                                  : launch_pass_t<double, T, 1, uint16_t>(a, s);
  return tbytes == 1 ? launch_pass_t<double, T, 2, uint8_t>(a, s)
                     : launch_pass_t<double, T, 2, uint16_t>(a, s);
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
    hipFuncSetAttribute((const void *)k_small<float>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute((const void *)k_small<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
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

hipError_t launch_scale_copy(int precision, const void *src, void *dst, uint64_t N, double re,
                             double im, hipStream_t s) {
  unsigned g = grid_for(N, 256);
  if (precision == 0)
    k_scale_copy<float><<<g, 256, 0, s>>>((const float2 *)src, (float2 *)dst, N, re, im);
  else
    k_scale_copy<double><<<g, 256, 0, s>>>((const double2 *)src, (double2 *)dst, N, re, im);
  return hipGetLastError();
}

}  // namespace qaoa
