// Mixers applied through their eigendecomposition (Golden et al., JuliQAOA, SC-W 2023,
// Sec. 2.1-2.2): the clique mixer sum_{i<j} X_iX_j + Y_iY_j, the ring mixer
// sum_i X_iX_{i+1} + Y_iY_{i+1} (i + 1 mod n), or any real symmetric matrix handed over by the
// caller. On the weight-k states (increasing integer order) the clique and ring mixers are
// real symmetric matrices H with entry 2 between states that differ by one allowed swap.
// H is diagonalised once in FP64 (H = V D V^T, rocSOLVER), and every round applies
//     psi <- exp(-i gamma C) psi,   psi <- V exp(-i beta D) V^T psi,
// i.e. two dense products per round, for all angle sets at once: the state of S angle sets is
// an N x 2S real matrix (real and imaginary parts as separate columns).
//
// FP32 form: each product is formed from FP16 halves with FP32 accumulation on the matrix
// cores, by the hand-written split-FP16 MFMA kernel of qaoa_gemm.hip: with
// x = x_hi + 2^-11 x_lo (x_hi = fp16(x), x_lo = fp16(2^11 (x - x_hi))),
//     V B ~ V_hi B_hi + 2^-11 (V_hi B_lo + V_lo B_hi)
// in one launch; the dropped V_lo B_lo term is 2^-22 relative. FP64 form: DGEMM on the FP64
// eigenbasis (rocBLAS).
//
// In the FP32 form every elementwise step (e^{-i beta D}, the next phase, <C>, lambda and the
// gradient sums) runs in the epilogue of the product that precedes it, on the product's tile
// in registers, and writes the next product's FP16 input directly (qaoa_gemm.hip).
//
// Gradient: the reverse sweep of the X path with H_M = V D V^T. The forward sweep keeps, per
// round, the phased state (before V^T) and its eigen-coefficients after exp(-i beta D); then
// only the adjoint vector needs products:
//   lam~ = V^T lam;  g_beta = 2 sum_r D_r Im(conj(lam~_r) phi~_r);  lam~ *= exp(+i beta D);
//   lam = V lam~;    g_gamma = 2 sum_x (C - c0) Im(conj(lam) phi);  lam *= exp(+i gamma C).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/qaoa.h"
#include "qaoa_clique.h"
#include "qaoa_internal.h"

namespace qaoa {

namespace {

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
  void *get(size_t bytes) {
    if (bytes <= cap && p) return p;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (bytes == 0) return nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw CliqueError{QAOA_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    cap = bytes;
    return p;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

void hipchk(hipError_t e, const char *what) {
  if (e != hipSuccess) throw CliqueError{QAOA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}
void blaschk(rocblas_status s, const char *what) {
  if (s != rocblas_status_success)
    throw CliqueError{QAOA_ERR_HIP, std::string(what) + ": " + rocblas_status_to_string(s)};
}

int64_t binom64(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

constexpr int RB_ROWS = 1024;  // rows per block in the elementwise kernels (4 per thread)

}  // namespace

struct CliqueMixer {
  int n = 0, k = 0;
  int64_t N = 0;
  int64_t Mp = 0, Kp = 0;  // rows / K of the padded FP16 planes (multiples of 256 / 128)
  rocblas_handle blas = nullptr;
  Buf V, D, V16;  // FP64 eigenbasis (N x N col-major, column j = eigenvector j), eigenvalues,
                  // FP16 planes [VT_hi, VT_lo, VN_hi, VN_lo], each Mp x Kp: row r of VT is
                  // eigenvector r (the V^T product), row x of VN is row x of V (the V product)
  Buf X, Y, B, B16, ckP, ckT, partials, params, luts, results, hres_dev;  // B: FP64 form's product input,
                                                                          // B16: FP32 form's (FP16 planes)
  Buf ws;               // the split-FP16 product's workspace (its XCD-balanced schedule)
  size_t b_zeroed = 0;  // bytes of B16 cleared since its allocation (its padding must stay zero)
  std::vector<double> hres;
  CliqueTimer timer;
  ~CliqueMixer() {
    if (blas) (void)rocblas_destroy_handle(blas);
  }
};

void CliqueMixerDeleter::operator()(CliqueMixer *m) const { delete m; }

void clique_set_timer(CliqueMixer &m, const CliqueTimer &t) { m.timer = t; }

// ---------------------------------------------------------------- kernels

// Rank of a weight-k integer y among the weight-k integers in increasing order
// (combinatorial number system: sum over its set bits b_1 < ... < b_k of C(b_i, i)).
__device__ int64_t rank_hw(uint64_t y, const int64_t *binom) {
  int64_t r = 0;
  int i = 1;
  for (int b = 0; b < 64 && y; b++) {
    if ((y >> b) & 1u) {
      r += binom[b * 33 + i];
      i++;
      y &= ~(1ull << b);
    }
  }
  return r;
}

// The r-th weight-k integer in increasing order.
__device__ uint64_t unrank_hw(int64_t r, int n, int k, const int64_t *binom) {
  uint64_t rem = (uint64_t)r, x = 0;
  int a = n - 1;
  for (int i = k; i >= 1; i--) {
    while (a >= i && (uint64_t)binom[a * 33 + i] > rem) a--;
    x |= 1ull << a;
    rem -= (uint64_t)binom[a * 33 + i];
    a--;
  }
  return x;
}

// H[c, r] = 2 for every swap neighbour c of state r (H zeroed beforehand): any 1-bit moved to
// any 0-bit (clique), or only across the ring edges (i, i + 1 mod n) (ring).
__global__ void k_clique_matrix(int n, int k, int ring, int64_t N, const int64_t *__restrict__ binom,
                                double *__restrict__ H) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const uint64_t x = unrank_hw(r, n, k, binom);
  for (int a = 0; a < n; a++) {
    if (!((x >> a) & 1u)) continue;
    for (int b = 0; b < n; b++) {
      if ((x >> b) & 1u) continue;
      if (ring && b != (a + 1) % n && a != (b + 1) % n) continue;
      const uint64_t y = x ^ (1ull << a) ^ (1ull << b);
      H[rank_hw(y, binom) + r * N] = 2.0;
    }
  }
}

// FP16 halves of V: hi = fp16(v), lo = fp16(2^11 (v - hi)), into the zero-padded fragment-major
// planes of the split products (VT: row r = eigenvector r; VN: row x = row x of V; rows of Kp).
__global__ void k_split_v(const double *__restrict__ V, int64_t N, int64_t Mp, int64_t Kp, __half *__restrict__ P) {
  const int64_t total = N * N, stride = (int64_t)gridDim.x * blockDim.x, plane = Mp * Kp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t x = i % N, r = i / N;  // V[x][r]: component x of eigenvector r
    const double v = V[i];
    const __half hi = __float2half((float)v);
    const __half lo = __float2half((float)((v - (double)__half2float(hi)) * 2048.0));
    const int64_t t = split_frag_offset(r, x, Kp), n = split_frag_offset(x, r, Kp);
    P[t] = hi;
    P[plane + t] = lo;
    P[2 * plane + n] = hi;
    P[3 * plane + n] = lo;
  }
}

template <typename R> struct CT;
template <> struct CT<float> { using T2 = float2; };
template <> struct CT<double> { using T2 = double2; };

// Write the complex value v of row x, set s as the next product's input. FP32 form: FP16
// halves in two blocked planes (lo plane at B, hi plane at B + plane halves; state column c is
// row c of the plane, rows of ldb halves); FP64 form: the value itself, column c at c * ldb.
template <typename R>
__device__ __forceinline__ void emit(void *B, int64_t ldb, int64_t plane, int64_t x, int s, R re, R im) {
  if constexpr (sizeof(R) == 4) {
    __half *b = (__half *)B;
    const __half hr = __float2half(re), hi = __float2half(im);
    const int64_t c0 = split_plane_offset(2 * s, x, ldb), c1 = split_plane_offset(2 * s + 1, x, ldb);
    b[plane + c0] = hr;
    b[c0] = __float2half((re - __half2float(hr)) * 2048.0f);
    b[plane + c1] = hi;
    b[c1] = __float2half((im - __half2float(hi)) * 2048.0f);
  } else {
    R *b = (R *)B;
    b[(int64_t)(2 * s) * ldb + x] = re;
    b[(int64_t)(2 * s + 1) * ldb + x] = im;
  }
}

template <typename TT>
__device__ __forceinline__ uint32_t cval(const void *t, int64_t x) {
  return (uint32_t)((const TT *)t)[x];
}

// Block sum of two doubles per thread (256 threads), written as partials.
__device__ void block_sum2(double a, double b, double *pa, double *pb) {
  __shared__ double ra[4], rb[4];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = a;
    rb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (pa) *pa = (ra[0] + ra[1]) + (ra[2] + ra[3]);
    if (pb) *pb = (rb[0] + rb[1]) + (rb[2] + rb[3]);
  }
}

// Initial state (uniform over the weight-k states, or the caller's) -> phase of round 1 ->
// next product's input (and the phased state kept for the gradient).
template <typename R>
__global__ void k_init(R *__restrict__ X, int64_t N, const void *psi0) {
  const int s = blockIdx.y;
  const R u = (R)(1.0 / sqrt((double)N));
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    R re = u, im = 0;
    if (psi0) {
      const typename CT<R>::T2 v = ((const typename CT<R>::T2 *)psi0)[x];
      re = v.x;
      im = v.y;
    }
    X[(int64_t)(2 * s) * N + x] = re;
    X[(int64_t)(2 * s + 1) * N + x] = im;
  }
}

// psi(x, s) *= LUT_s[C(x)]; keep the result (ck) and emit it for V^T.
template <typename R, typename TT>
__global__ void k_phase(const R *__restrict__ X, int64_t N, const void *table,
                        const typename CT<R>::T2 *__restrict__ luts, int lut_len, R *ck, void *B, int64_t ldb,
                        int64_t plane) {
  const int s = blockIdx.y;
  const typename CT<R>::T2 *L = luts + (int64_t)s * lut_len;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const R a = X[(int64_t)(2 * s) * N + x], b = X[(int64_t)(2 * s + 1) * N + x];
    const typename CT<R>::T2 l = L[cval<TT>(table, x)];
    const R re = a * l.x - b * l.y, im = a * l.y + b * l.x;
    if (ck) {
      ck[(int64_t)(2 * s) * N + x] = re;
      ck[(int64_t)(2 * s + 1) * N + x] = im;
    }
    emit<R>(B, ldb, plane, x, s, re, im);
  }
}

// Eigen-coefficients t(r, s) (product output Y) times exp(sign i beta_s D_r), phase in FP64.
// With tref: g_beta partial sum_r D_r Im(conj(t) tref) before the phase (one per block).
template <typename R>
__global__ __launch_bounds__(256) void k_eig(const R *__restrict__ Y, int64_t N, const double *__restrict__ D,
                                             const double *__restrict__ betas, double sign,
                                             const R *tref, R *ck, void *B, int64_t ldb, int64_t plane,
                                             double *gpart, int nblk) {
  const int s = blockIdx.y;
  const double beta = betas[s];
  double acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RB_ROWS;
  for (int64_t r = r0 + threadIdx.x; r < N && r < r0 + RB_ROWS; r += 256) {
    const R a = Y[(int64_t)(2 * s) * N + r], b = Y[(int64_t)(2 * s + 1) * N + r];
    const double d = D[r];
    if (tref) {
      const R ta = tref[(int64_t)(2 * s) * N + r], tb = tref[(int64_t)(2 * s + 1) * N + r];
      acc += d * ((double)a * tb - (double)b * ta);
    }
    double sn, cs;
    sincos(sign * beta * d, &sn, &cs);
    const R re = (R)((double)a * cs - (double)b * sn), im = (R)((double)a * sn + (double)b * cs);
    if (ck) {
      ck[(int64_t)(2 * s) * N + r] = re;
      ck[(int64_t)(2 * s + 1) * N + r] = im;
    }
    emit<R>(B, ldb, plane, r, s, re, im);
  }
  if (gpart) block_sum2(acc, 0.0, gpart + (int64_t)s * nblk + blockIdx.x, nullptr);
}

// E and Nrm partials of the final state.
template <typename R, typename TT>
__global__ __launch_bounds__(256) void k_expect(const R *__restrict__ X, int64_t N, const void *table,
                                                const double *__restrict__ vals, double *epart, double *npart,
                                                int nblk) {
  const int s = blockIdx.y;
  double e = 0.0, nr = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RB_ROWS;
  for (int64_t x = r0 + threadIdx.x; x < N && x < r0 + RB_ROWS; x += 256) {
    const double a = X[(int64_t)(2 * s) * N + x], b = X[(int64_t)(2 * s + 1) * N + x];
    const double pr = a * a + b * b;
    e += pr * vals[cval<TT>(table, x)];
    nr += pr;
  }
  block_sum2(e, nr, epart + (int64_t)s * nblk + blockIdx.x, npart + (int64_t)s * nblk + blockIdx.x);
}

// lam = (C - c0) psi_p, emitted for V^T.
template <typename R, typename TT>
__global__ void k_lambda(const R *__restrict__ X, int64_t N, const void *table, const double *__restrict__ vals,
                         double c0, void *B, int64_t ldb, int64_t plane) {
  const int s = blockIdx.y;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const R k = (R)(vals[cval<TT>(table, x)] - c0);
    emit<R>(B, ldb, plane, x, s, k * X[(int64_t)(2 * s) * N + x], k * X[(int64_t)(2 * s + 1) * N + x]);
  }
}

// g_gamma partial sum_x (C - c0) Im(conj(lam) phi) with phi the kept phased state; then
// lam *= LUT_s[C] (inverse phase) and emit it for the next V^T (if B).
template <typename R, typename TT>
__global__ __launch_bounds__(256) void k_gamma(const R *__restrict__ L, int64_t N, const void *table,
                                               const double *__restrict__ vals, double c0, const R *__restrict__ phi,
                                               const typename CT<R>::T2 *luts, int lut_len, void *B,
                                               int64_t ldb, int64_t plane, double *gpart, int nblk) {
  const int s = blockIdx.y;
  double acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RB_ROWS;
  for (int64_t x = r0 + threadIdx.x; x < N && x < r0 + RB_ROWS; x += 256) {
    const R a = L[(int64_t)(2 * s) * N + x], b = L[(int64_t)(2 * s + 1) * N + x];
    const R pa = phi[(int64_t)(2 * s) * N + x], pb = phi[(int64_t)(2 * s + 1) * N + x];
    const uint32_t c = cval<TT>(table, x);
    acc += (vals[c] - c0) * ((double)a * pb - (double)b * pa);
    if (B) {
      const typename CT<R>::T2 l = luts[(int64_t)s * lut_len + c];
      emit<R>(B, ldb, plane, x, s, a * l.x - b * l.y, a * l.y + b * l.x);
    }
  }
  block_sum2(acc, 0.0, gpart + (int64_t)s * nblk + blockIdx.x, nullptr);
}

template <typename R>
__global__ void k_export(const R *__restrict__ X, int64_t N, typename CT<R>::T2 *out) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x)
    out[x] = typename CT<R>::T2{X[x], X[N + x]};
}

// ---------------------------------------------------------------- setup

std::unique_ptr<CliqueMixer, CliqueMixerDeleter> clique_create(int kind, int n, int k, const double *host_matrix,
                                                                 const double *host_eigenvalues, hipStream_t st) {
  std::unique_ptr<CliqueMixer, CliqueMixerDeleter> m(new CliqueMixer());
  m->n = n;
  m->k = k;
  const int64_t N = k < 0 ? (int64_t(1) << n) : binom64(n, k);
  m->N = N;
  blaschk(rocblas_create_handle(&m->blas), "rocblas_create_handle");
  blaschk(rocblas_set_stream(m->blas, st), "rocblas_set_stream");
  // clique matrix (FP64, dense) -> eigendecomposition in place
  double *H = (double *)m->V.get((size_t)N * N * sizeof(double));
  double *Dv = (double *)m->D.get((size_t)N * sizeof(double));
  std::vector<int64_t> hb(33 * 33);
  for (int a = 0; a <= 32; a++)
    for (int b = 0; b <= 32; b++) hb[a * 33 + b] = binom64(a, b);
  Buf dbin, E, info;
  int64_t *db = (int64_t *)dbin.get(hb.size() * sizeof(int64_t));
  hipchk(hipMemcpyAsync(db, hb.data(), hb.size() * sizeof(int64_t), hipMemcpyHostToDevice, st), "binom upload");
  if (kind == MIX_EIGEN) {
    // a stored eigendecomposition: V (column j = eigenvector j) and D, no eigensolver
    hipchk(hipMemcpyAsync(H, host_matrix, (size_t)N * N * sizeof(double), hipMemcpyHostToDevice, st), "V upload");
    hipchk(hipMemcpyAsync(Dv, host_eigenvalues, (size_t)N * sizeof(double), hipMemcpyHostToDevice, st), "D upload");
  } else if (kind == MIX_MATRIX) {
    hipchk(hipMemcpyAsync(H, host_matrix, (size_t)N * N * sizeof(double), hipMemcpyHostToDevice, st), "matrix upload");
  } else {
    hipchk(hipMemsetAsync(H, 0, (size_t)N * N * sizeof(double), st), "clear H");
    k_clique_matrix<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, k, kind == MIX_RING ? 1 : 0, N, db, H);
    hipchk(hipGetLastError(), "k_clique_matrix");
  }
  if (kind != MIX_EIGEN) {
    double *dE = (double *)E.get((size_t)N * sizeof(double));
    rocblas_int *dinfo = (rocblas_int *)info.get(sizeof(rocblas_int));
    blaschk(rocsolver_dsyevd(m->blas, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)N, H,
                             (rocblas_int)N, Dv, dE, dinfo),
            "rocsolver_dsyevd");
    rocblas_int hinfo = 0;
    hipchk(hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, st), "info download");
    hipchk(hipStreamSynchronize(st), "eigendecomposition");
    if (hinfo != 0) throw CliqueError{QAOA_ERR_HIP, "eigendecomposition did not converge"};
  }
  // FP16 halves for the FP32 form, in zero-padded planes
  m->Mp = (N + SPLIT_MTILE - 1) / SPLIT_MTILE * SPLIT_MTILE;
  m->Kp = (N + SPLIT_KQUANT - 1) / SPLIT_KQUANT * SPLIT_KQUANT;
  const size_t vbytes = (size_t)4 * m->Mp * m->Kp * sizeof(__half);
  __half *P16 = (__half *)m->V16.get(vbytes);
  hipchk(hipMemsetAsync(P16, 0, vbytes, st), "clear FP16 planes");
  k_split_v<<<4096, 256, 0, st>>>(H, N, m->Mp, m->Kp, P16);
  hipchk(hipGetLastError(), "k_split_v");
  hipchk(hipStreamSynchronize(st), "split V");
  return m;
}

void clique_export(const CliqueMixer &m, double *host_V, double *host_D, hipStream_t st) {
  const size_t N = (size_t)m.N;
  hipchk(hipMemcpyAsync(host_V, m.V.p, N * N * sizeof(double), hipMemcpyDeviceToHost, st), "V download");
  hipchk(hipMemcpyAsync(host_D, m.D.p, N * sizeof(double), hipMemcpyDeviceToHost, st), "D download");
  hipchk(hipStreamSynchronize(st), "eigenbasis download");
}

int64_t clique_size(const CliqueMixer &m) { return m.N; }

// ---------------------------------------------------------------- evaluation

namespace {

template <typename R>
struct Dense {
  CliqueMixer &m;
  hipStream_t st;
  int64_t N;
  int cols;       // 2S
  int64_t ldb;    // column stride of the product input B (Kp halves for FP32, N for FP64)
  int64_t plane;  // FP32: halves between the lo and hi planes of B

  // FP64 form: out (N x cols, ld N) = op(V) in (the product input B), op = V^T (transpose) or
  // V, on the FP64 eigenbasis (the FP32 form's products carry their epilogues, run_clique)
  void product(bool transpose, const void *B, R *out) {
    static_assert(sizeof(R) == 8, "the FP32 form multiplies through launch_split_gemm_epi");
    if (m.timer.begin) m.timer.begin(m.timer.ctx, st);
    const rocblas_int n = (rocblas_int)N, c = cols;
    const double one = 1.0, zero = 0.0;
    blaschk(rocblas_set_stream(m.blas, st), "rocblas_set_stream");
    blaschk(rocblas_dgemm(m.blas, transpose ? rocblas_operation_transpose : rocblas_operation_none,
                          rocblas_operation_none, n, c, n, &one, (const double *)m.V.p, n, (const double *)B, n,
                          &zero, out, n),
            "rocblas_dgemm");
    // algorithmic work of one real N x N x cols product
    if (m.timer.end) m.timer.end(m.timer.ctx, st, QAOA_KC_DENSE, 0.0, 2.0 * (double)N * N * cols);
  }
};

template <typename R, typename TT>
void run_clique(CliqueMixer &m, const CliqueEval &ev, int p, const double *angles, int S, const void *d_psi0,
                int grad, double *out_expect, double *out_grad, void *d_state, hipStream_t st) {
  using T2 = typename CT<R>::T2;
  const int64_t N = m.N;
  const int cols = 2 * S;
  const size_t mat = (size_t)N * cols * sizeof(R);
  R *X = (R *)m.X.get(mat);
  R *Y = sizeof(R) == 4 ? nullptr : (R *)m.Y.get(mat);  // the FP32 form keeps no product output
  // product input: FP32 form, lo and hi FP16 planes of Ncp = roundup(cols, 128) columns of Kp
  // halves (the padding rows and columns stay zero); FP64 form, N x cols doubles
  const int64_t ncp = ((int64_t)cols + SPLIT_TILE - 1) / SPLIT_TILE * SPLIT_TILE;
  const int64_t ldb = sizeof(R) == 4 ? m.Kp : N, plane = sizeof(R) == 4 ? ncp * m.Kp : 0;
  // FP32 form: two sets of planes, the input of the current product and the one its epilogue
  // writes (ping-pong)
  const size_t bbytes = sizeof(R) == 4 ? (size_t)2 * 2 * ncp * m.Kp * sizeof(__half) : mat;
  // the FP16 planes have their own buffer: its padding is written by nothing but this clear
  Buf &bb = sizeof(R) == 4 ? m.B16 : m.B;
  const void *bold = bb.p;
  void *B = bb.get(bbytes);
  if (sizeof(R) == 4 && (B != bold || m.b_zeroed < bbytes)) {
    hipchk(hipMemsetAsync(B, 0, bb.cap, st), "clear product input");
    m.b_zeroed = bb.cap;
  }
  R *ckP = grad ? (R *)m.ckP.get(mat * p) : nullptr;
  R *ckT = grad ? (R *)m.ckT.get(mat * p) : nullptr;
  // partial sums per block of rows: the elementwise kernels' blocks (FP64 form) or the
  // product's row tiles (FP32 form: the reductions are fused into the product epilogues)
  const int nblk = sizeof(R) == 4 ? (int)((N + SPLIT_MTILE - 1) / SPLIT_MTILE) : (int)((N + RB_ROWS - 1) / RB_ROWS);
  const int nout = 2 + 2 * p;
  double *part = (double *)m.partials.get((size_t)nout * S * nblk * sizeof(double));
  auto pslot = [&](int o) { return part + (size_t)o * S * nblk; };
  // parameters: betas [p][S], LUT jobs (forward, inverse) [2p][S], contribution counts
  std::vector<double> betas((size_t)p * S);
  std::vector<LutJob> jobs((size_t)2 * p * S);
  for (int s = 0; s < S; s++)
    for (int k = 0; k < p; k++) {
      betas[(size_t)k * S + s] = angles[(size_t)s * 2 * p + k];
      const double g = angles[(size_t)s * 2 * p + p + k];
      jobs[(size_t)k * S + s] = LutJob{g, 1.0, 0.0, -1.0};
      jobs[(size_t)(p + k) * S + s] = LutJob{g, 1.0, 0.0, 1.0};
    }
  std::vector<int> cnt(nout, 1);
  const size_t b_bytes = betas.size() * sizeof(double), j_bytes = jobs.size() * sizeof(LutJob);
  const size_t off_j = (b_bytes + 255) & ~size_t(255), off_c = (off_j + j_bytes + 255) & ~size_t(255);
  const size_t total = off_c + nout * sizeof(int);
  std::vector<unsigned char> h(total);
  std::memcpy(h.data(), betas.data(), b_bytes);
  std::memcpy(h.data() + off_j, jobs.data(), j_bytes);
  std::memcpy(h.data() + off_c, cnt.data(), nout * sizeof(int));
  unsigned char *d = (unsigned char *)m.params.get(total);
  hipchk(hipMemcpyAsync(d, h.data(), total, hipMemcpyHostToDevice, st), "parameter upload");
  const double *dbeta = (const double *)d;
  T2 *dluts = (T2 *)m.luts.get(jobs.size() * (size_t)ev.lut_len * sizeof(T2));
  hipchk(launch_luts(sizeof(R) == 4 ? 0 : 1, (const LutJob *)(d + off_j), (int)jobs.size(), ev.lut_len, ev.vals,
                     dluts, st),
         "LUTs");
  auto lut_f = [&](int k) { return dluts + (size_t)k * S * ev.lut_len; };
  auto lut_b = [&](int k) { return dluts + (size_t)(p + k) * S * ev.lut_len; };

  Dense<R> dense{m, st, N, cols, ldb, plane};
  const dim3 eg((unsigned)((N + 255) / 256 < 1024 ? (N + 255) / 256 : 1024), (unsigned)S);
  const dim3 rg((unsigned)nblk, (unsigned)S);
  auto launched = [&](const char *w) { hipchk(hipGetLastError(), w); };
  auto tbegin = [&]() {
    if (m.timer.begin) m.timer.begin(m.timer.ctx, st);
  };
  auto tend = [&](double bytes) {
    if (m.timer.end) m.timer.end(m.timer.ctx, st, QAOA_KC_OTHER, bytes, 0.0);
  };

  if constexpr (sizeof(R) == 4) {
    // FP32 form: every elementwise step runs in the epilogue of the product before it
    const int64_t bp = (int64_t)2 * plane;  // halves per set of planes
    _Float16 *Bset[2] = {(_Float16 *)B, (_Float16 *)B + bp};
    int cur = 0;
    const __half *P16 = (const __half *)m.V16.p;
    const int64_t vp = m.Mp * m.Kp;
    const size_t wsb = split_gemm_ws_bytes((int)N, cols, m.Kp);
    float *dws = wsb ? (float *)m.ws.get(wsb) : nullptr;
    auto product = [&](bool transpose, int mode, SplitEpi e) {
      const __half *mh = transpose ? P16 : P16 + 2 * vp, *ml = mh + vp;
      const _Float16 *bl = Bset[cur], *bh = bl + plane;
      e.bld = m.Kp;
      e.bplane = plane;
      e.ldc = N;
      e.D = (const double *)m.D.p;
      e.table = ev.table;
      e.tbytes = ev.tbytes;
      e.vals = ev.vals;
      e.c0 = ev.c0;
      e.lut_len = ev.lut_len;
      e.nblk = nblk;
      e.ws = dws;
      if (m.timer.begin) m.timer.begin(m.timer.ctx, st);
      hipchk(launch_split_gemm_epi(mode, bh, bl, mh, ml, m.Kp, (int)N, cols, e, st), "split-FP16 product");
      if (m.timer.end) m.timer.end(m.timer.ctx, st, QAOA_KC_DENSE, 0.0, 2.0 * (double)N * N * cols);
      cur ^= 1;
    };
    tbegin();
    k_init<R><<<eg, 256, 0, st>>>(X, N, d_psi0);
    launched("k_init");
    k_phase<R, TT><<<eg, 256, 0, st>>>(X, N, ev.table, lut_f(0), ev.lut_len, grad ? ckP : nullptr, Bset[cur], ldb,
                                        plane);
    launched("k_phase");
    tend((double)mat * (grad ? 4 : 3));
    for (int k = 0; k < p; k++) {
      SplitEpi e{};
      e.bout = Bset[cur ^ 1];
      e.betas = dbeta + (size_t)k * S;
      e.ck = grad ? (float *)(ckT + (size_t)k * N * cols) : nullptr;
      product(true, SE_EIG, e);
      SplitEpi f{};
      f.bout = Bset[cur ^ 1];
      if (k + 1 < p) {
        f.luts = (const float2 *)lut_f(k + 1);
        f.ck = grad ? (float *)(ckP + (size_t)(k + 1) * N * cols) : nullptr;
        product(false, SE_PHASE, f);
      } else {
        f.C = (float *)X;
        f.part0 = pslot(0);
        f.part1 = pslot(1);
        if (!grad) f.bout = nullptr;
        product(false, SE_LAST, f);
      }
    }
    if (d_state) {
      k_export<R><<<eg.x, 256, 0, st>>>(X, N, (T2 *)d_state);
      launched("k_export");
    }
    if (grad) {
      // lambda = (C - c0) psi_p was emitted by the last forward product
      for (int k = p - 1; k >= 0; k--) {
        SplitEpi e{};
        e.bout = Bset[cur ^ 1];
        e.betas = dbeta + (size_t)k * S;
        e.ckr = (const float *)(ckT + (size_t)k * N * cols);
        e.part0 = pslot(2 + k);
        product(true, SE_REIG, e);
        SplitEpi f{};
        f.bout = k > 0 ? Bset[cur ^ 1] : nullptr;
        f.luts = (const float2 *)lut_b(k);
        f.ckr = (const float *)(ckP + (size_t)k * N * cols);
        f.part0 = pslot(2 + p + k);
        product(false, SE_RPHASE, f);
      }
    }
  } else {
    // forward sweep
    tbegin();
    k_init<R><<<eg, 256, 0, st>>>(X, N, d_psi0);
    launched("k_init");
    tend((double)mat);
    for (int k = 0; k < p; k++) {
      tbegin();
      k_phase<R, TT><<<eg, 256, 0, st>>>(X, N, ev.table, lut_f(k), ev.lut_len, grad ? ckP + (size_t)k * N * cols : nullptr, B,
                                          ldb, plane);
      launched("k_phase");
      tend((double)mat * (grad ? 3 : 2));
      dense.product(true, B, Y);
      tbegin();
      k_eig<R><<<rg, 256, 0, st>>>(Y, N, m.D.p ? (const double *)m.D.p : nullptr, dbeta + (size_t)k * S, -1.0, nullptr,
                                   grad ? ckT + (size_t)k * N * cols : nullptr, B, ldb, plane, nullptr, nblk);
      launched("k_eig");
      tend((double)mat * (grad ? 3 : 2));
      dense.product(false, B, X);
    }
    tbegin();
    k_expect<R, TT><<<rg, 256, 0, st>>>(X, N, ev.table, ev.vals, pslot(0), pslot(1), nblk);
    launched("k_expect");
    tend((double)mat);
    if (d_state) {
      k_export<R><<<eg.x, 256, 0, st>>>(X, N, (T2 *)d_state);
      launched("k_export");
    }
    // reverse sweep (only the adjoint vector is multiplied; phi comes from the forward keeps)
    if (grad) {
      k_lambda<R, TT><<<eg, 256, 0, st>>>(X, N, ev.table, ev.vals, ev.c0, B, ldb, plane);
      launched("k_lambda");
      for (int k = p - 1; k >= 0; k--) {
        dense.product(true, B, Y);
        tbegin();
        k_eig<R><<<rg, 256, 0, st>>>(Y, N, (const double *)m.D.p, dbeta + (size_t)k * S, 1.0,
                                     ckT + (size_t)k * N * cols, nullptr, B, ldb, plane, pslot(2 + k), nblk);
        launched("k_eig");
        tend((double)mat * 3);
        dense.product(false, B, X);
        tbegin();
        k_gamma<R, TT><<<rg, 256, 0, st>>>(X, N, ev.table, ev.vals, ev.c0, ckP + (size_t)k * N * cols, lut_b(k), ev.lut_len,
                                           k > 0 ? B : nullptr, ldb, plane, pslot(2 + p + k), nblk);
        launched("k_gamma");
        tend((double)mat * 3);
      }
    }
  }
  // fixed-order reduction of the partials: out[s][o]
  double *dres = (double *)m.results.get((size_t)S * nout * sizeof(double));
  hipchk(launch_finalize(part, (const int *)(d + off_c), 1, S, nblk, nout, dres, st), "finalize");
  m.hres.resize((size_t)S * nout);
  hipchk(hipMemcpyAsync(m.hres.data(), dres, (size_t)S * nout * sizeof(double), hipMemcpyDeviceToHost, st),
         "result download");
  hipchk(hipStreamSynchronize(st), "constrained evaluation");
  for (int s = 0; s < S; s++) {
    const double *r = m.hres.data() + (size_t)s * nout;
    const double E = r[0], Nr = r[1];
    if (out_expect) out_expect[s] = E / Nr;
    if (grad && out_grad)
      for (int k = 0; k < 2 * p; k++) out_grad[(size_t)s * 2 * p + k] = 2.0 * r[2 + k] / Nr;
  }
}

}  // namespace

void clique_evaluate(CliqueMixer &m, const CliqueEval &ev, int p, const double *angles, int nsets,
                     const void *d_psi0, int precision, int grad, double *out_expect, double *out_grad,
                     void *d_state, hipStream_t st) {
  if (ev.N != m.N) throw CliqueError{QAOA_ERR_INVALID_ARG, "problem size differs from the mixer's subspace"};
  if (d_state && nsets != 1) throw CliqueError{QAOA_ERR_INVALID_ARG, "state output needs one angle set"};
  if (precision == QAOA_FP32) {
    if (ev.tbytes == 1) run_clique<float, uint8_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
    else run_clique<float, uint16_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
  } else {
    if (ev.tbytes == 1) run_clique<double, uint8_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
    else run_clique<double, uint16_t>(m, ev, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
  }
}

}  // namespace qaoa
