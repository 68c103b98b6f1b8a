// Internal declarations shared by the HIP kernels (qaoa_kernels.hip) and the host runtime
// (qaoa_api.cpp). Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace qaoa {

// Tile of the X-mixer pass kernels: 2^T amplitudes per workgroup, 256 threads, 2^(T-8)
// amplitudes per thread and vector held in registers. FP32 uses T=13 (64 KiB of complex64
// per vector), FP64 uses T=12 (64 KiB of complex128).
constexpr int TILE_BITS_F32 = 13;
constexpr int TILE_BITS_F64 = 12;
constexpr int PASS_THREADS = 256;
// Shortest run of contiguous amplitudes a strided tile keeps together (256 B either way).
constexpr int MIN_CONTIG_F32 = 5;
constexpr int MIN_CONTIG_F64 = 4;
// Shortest run a strided tile may take when that saves a whole tile of the cover (64 B either
// way: n = 30..33 in FP32 and 29..32 in FP64 then need three tiles instead of four).
constexpr int MIN_CONTIG_NARROW_F32 = 3;
constexpr int MIN_CONTIG_NARROW_F64 = 2;
// Whole-state (one workgroup per item) kernel: both vectors resident in LDS.
constexpr int SMALL_MAX_N_F32 = 13;
constexpr int SMALL_MAX_N_F64 = 12;
constexpr int SMALL_THREADS = 256;
// Largest phase lookup table the kernels stage in LDS: the cost table stores, per state, the
// index of its value among at most MAX_LUT distinct values (a graph table's index is the
// value itself).
constexpr int MAX_LUT = 1024;

// Pass flags (X-mixer tile passes). A pass runs: load, part 1 (register stages H, M, L),
// middle (elementwise steps at the end of part 1), part 2 (stages L, M, H), store.
enum : uint32_t {
  PF_GEN_PHI = 1u << 0,      // phi <- uniform amplitude u0 instead of loading
  PF_LOAD_PSI0 = 1u << 1,    // phi <- caller's initial state (natural layout)
  PF_LOAD_PHI = 1u << 2,
  PF_LOAD_LAM = 1u << 3,
  PF_EXPECT = 1u << 4,       // middle: E += |phi|^2 C, N += |phi|^2
  PF_LAMBDA = 1u << 5,       // middle: lam <- rho (C - c0) phi
  PF_GGAMMA = 1u << 6,       // middle: += w Im(conj(lam) C phi)
  PF_PHASE = 1u << 7,        // middle: phi *= LUT[C]
  PF_STORE_PHI = 1u << 8,
  PF_STORE_LAM = 1u << 9,
  PF_XT1 = 1u << 10,         // part 1: X-pair terms of each rotated bit, before rotating it
  PF_XT2 = 1u << 11,         // part 2: same
  PF_ROT1_BOTH = 1u << 12,   // part 1 also rotates lam
  PF_ROT2_BOTH = 1u << 13,   // part 2 also rotates lam
  PF_PHASE_BOTH = 1u << 14,  // the phase also applies to lam
  PF_SCALE_OUT = 1u << 15,   // (unused)
  PF_LOAD_SCALE = 1u << 16,  // phi *= (out_re + i out_im) right after loading
};

// Diagonal of a step of the X-product / multi-angle path: where the value index of basis
// state y comes from.
enum { XD_TABLE = 0, XD_POPCOUNT = 1, XD_TERMS = 2, XD_QUBIT = 3 };
constexpr int XD_MAX_TERMS = 10;
struct XDiag {
  int mode;             // XD_*
  int tbytes;           // XD_TABLE: 1 or 2
  const void *table;    // XD_TABLE: index table (2^n entries)
  int nterms;           // XD_TERMS: index bit t = parity of (y & masks[t])
  uint64_t masks[XD_MAX_TERMS];
};

// Partial-sum slots of one pass.
enum { SL_A = 0, SL_B = 1, SL_C = 2, NSLOT = 3 };

// Per (pass, angle set) parameters, read by every workgroup of the set.
template <typename R>
struct SetParams {
  R tau1, tau2;          // rotation parameter of part 1 / part 2
  double w1, w2;         // inner-product weight at the start of part 1 / part 2
  R lam_rho;             // lambda = lam_rho * (C - c0) * phi
  R out_re, out_im;      // load scale of phi (PF_LOAD_SCALE)
  int lut;               // index of this set's LUT in the LUT array (-1: none)
  int tflip;             // 1: the stored vector is the state with every bit flipped at this
                         // pass's elementwise steps, so they read C(~x) (the reversed table)
};

// Pass descriptor (kernel argument). Geometry: tile bits [0,c) are address bits [0,c);
// tile bits [c,T) are address bits [h0, h0+T-c); a workgroup's remaining address bits are
// [c,h0) and [h0+T-c, n), filled from its tile index r.
template <typename R>
struct PassArgs {
  int n, c, h0;
  uint32_t nwg;            // tiles per vector = 2^(n-T)
  int xcd_remap;           // give each XCD a contiguous range of tiles
  int nsets;               // angle sets (grid.y)
  uint64_t vstride;        // elements between consecutive sets' vectors
  void *phi, *lam;         // phi is read from `phi`, written to `phi_out` (equal: in place)
  void *phi_out;
  const void *psi0;        // natural layout, shared by all sets
  const void *table;       // tile-major table of this geometry: table[r * 2^T + e]
  const void *table_rev;   // the same array reversed (C(~x)); equal to table when C(~x) = C(x)
  const void *vals;        // R[lut_len]: cost value of each table index
  const void *luts;        // lut_len complex<R> entries per LUT
  int lut_len;
  uint32_t flags;
  uint32_t mask1, mask2;   // tile bits rotated in part 1 / part 2
  R u0;                    // uniform initial amplitude
  R lam_c0;
  const SetParams<R> *sp;  // [nsets]
  double *partials;        // slot s of set q, tile b: partials[slot_off[s] + q * nwg + b]
  int64_t slot_off[NSLOT]; // -1: slot unused
  // X-product passes whose middle is a parity-mask diagonal: index bit k = parity(y & xmasks[k]);
  // xreg[j] = the index of register j's part of y in the middle's register assignment
  uint64_t xmasks[XD_MAX_TERMS];
  int xnterms;
  uint16_t xreg[32];
  // Per-qubit multi-angle passes: vals holds, per angle set, 33 complex doubles (the constant
  // factor, then e^{+-2i beta_q} per qubit q); the LUT holds the register parts' factors. In
  // the reverse sweep the sum over all states goes to slot ma_total and the sum over the states
  // with bit q set to slot ma_slot + q * ma_stride; ma_src[q] says where bit q sits in the
  // middle's register assignment: register bit b (0..7), thread bit i (8 + i), or the tile
  // index (16).
  int64_t ma_total, ma_slot, ma_stride;
  int8_t ma_src[32];
  // State layout: swz == 0 stores element x of a vector at x; swz > 0 at
  // x ^ (((x >> swz_src) & 1023) << swz) (the top ten index bits folded into ten middle ones;
  // requires swz + 10 <= swz_src). Passes that read the caller's initial state (natural order)
  // run swz == 0.
  int swz, swz_src;
  int swz_add;  // 1: the tile's own address bits all lie below swz_src (uniform swizzle value)
  int cached;   // state loads and stores through the caches instead of non-temporal
};

// LUT construction job: luts[i][c] = scale_i * exp(sign_i * i * gamma_i * vals[c]),
// c < lut_len.
struct LutJob {
  double gamma, sre, sim, sign;
};

// Whole-state kernel item: one workgroup evolves one (problem, angle set) pair.
struct SmallItem {
  const void *table;    // device table (2^n entries), uint8 or uint16
  const double *vals;   // cost value of each table index (lut_len entries)
  int n;
  int tbytes;           // 1 or 2
  int sym;              // 1: C(~x) = C(x) for every x (flipped states read the table as is)
  int lut_len;          // number of table indices (largest index + 1)
  int angle_set;        // row of the angle array
  double c0;            // centre of lambda = (C - c0) psi
  int out_index;        // output row: out[out_index * (1 + 2p) + ...]
};

// Grover-mixer evaluation on the distinct cost values: one workgroup per item, classes held in
// registers (GROVER_CPT per thread, at most 256 * GROVER_CPT classes).
constexpr int GROVER_CPT = 8;
constexpr int GROVER_MAX_CLASSES = 256 * GROVER_CPT;
struct GroverItem {
  const double *vals;    // class values (nclass)
  const double *counts;  // degeneracy of each class (FP64, exact below 2^53)
  int nclass;
  int angle_set;         // row of the angle array
  int out_index;         // output row: out[out_index * (1 + 2p) + ...]
  double total;          // number of feasible states
  double c0;             // centre of lambda = (C - c0) psi
  double2 *amp_out;      // optional: final class amplitudes (nclass)
};

// ---------------------------------------------------------------- launch wrappers
hipError_t launch_cost_table_full(int n, int m, const int32_t *du, const int32_t *dv,
                                  const int32_t *dw, void *table, int tbytes, hipStream_t s);
hipError_t launch_cost_table_hw(int n, int k, int m, const int32_t *du, const int32_t *dv,
                                const int32_t *dw, const int64_t *dbinom, uint64_t N,
                                void *table, int tbytes, hipStream_t s);
hipError_t launch_table_max(const void *table, int tbytes, uint64_t N, unsigned *dmax,
                            hipStream_t s);
hipError_t launch_table_relayout(const void *src, void *dst, int tbytes, int n, int T, int c,
                                 int h0, hipStream_t s);
hipError_t launch_table_widen(const void *src, int tbytes, int64_t *dst, uint64_t N,
                              hipStream_t s);
hipError_t launch_luts(int precision, const LutJob *jobs, int njobs, int lut_len, const double *vals,
                       void *luts, hipStream_t s);
// dst[i] = src[count - 1 - i] (tables of 1 or 2 bytes per entry)
hipError_t launch_table_reverse(const void *src, void *dst, int tbytes, uint64_t count, hipStream_t s);
// dst[x] = vals[table[x]]
hipError_t launch_table_values(const void *table, int tbytes, const double *vals, double *dst, uint64_t N,
                               hipStream_t s);
// kind: 1 = forward pass (phi), 2 = reverse-sweep pass (phi, lam), 4 = reverse-sweep pass reading
// phi from a checkpoint (phi never stored), 3 = fused end of the
// forward sweep and start of the reverse sweep. sx: register stages holding the tile's
// rotated bits (bit 0: H, bit 1: M, bit 2: L; 7, 5, 3 or 1). shape: 0 = part 1 only,
// 1 = both parts with the kind's elementwise steps between them, 2 = phase then part 2
// (first forward pass), 3 = part 1 then a reduction (forward: <C>; reverse: gamma gradient).
hipError_t launch_pass_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes,
                           hipStream_t s);
hipError_t launch_pass_f64(const PassArgs<double> &a, int kind, int sx, int shape, int tbytes,
                           hipStream_t s);
// The same passes in the swizzled layout (a.swz > 0; qaoa_swz_f32.hip, qaoa_swz_f64.hip): stage
// set 7 only, no caller initial state; the access form follows a.cached and a.swz_add.
hipError_t launch_pass_swz_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes,
                               hipStream_t s);
hipError_t launch_pass_swz_f64(const PassArgs<double> &a, int kind, int sx, int shape, int tbytes,
                               hipStream_t s);
// The same passes with Y rotations and no X-pair terms (X-product mixers, qaoa_xpass.hip):
// kinds 1 (shapes 0, 1, 2, 3), 3 (shape 1), 2 and 4 (shapes 0, 1, 3); mixd (kinds 1, 2, 4, shape 1):
// 0 = the middle's diagonal is the cost's, XD_POPCOUNT / XD_TERMS = the mixer's, indexed by the
// Hamming weight of the state index / by its parities against PassArgs::xmasks.
hipError_t launch_hpass_f32(const PassArgs<float> &a, int kind, int sx, int shape, int tbytes, int mixd,
                           hipStream_t s);
hipError_t launch_hpass_f64(const PassArgs<double> &a, int kind, int sx, int shape, int tbytes, int mixd,
                           hipStream_t s);
hipError_t launch_finalize(const double *partials, const int *cnt, int maxc, int nsets,
                           int64_t nwg, int nout, double *out, hipStream_t s);
// stage != 0 (launch_small, launch_whole): each workgroup first copies its angle set into LDS, so
// items and angles may sit in mapped host memory (read once per workgroup, no copy beforehand).
hipError_t launch_small(int precision, const SmallItem *items, int n_items, int max_n,
                        int max_tbytes, int max_lut, const double *angles, int p, int grad,
                        double *out, hipStream_t s, int stage = 0);
// Index of the diagonal value of basis state y (XD_TABLE, XD_POPCOUNT, XD_TERMS).
__device__ __forceinline__ uint32_t xdiag_index(const XDiag &d, uint64_t y) {
  if (d.mode == XD_TABLE)
    return d.tbytes == 1 ? (uint32_t)((const uint8_t *)d.table)[y] : (uint32_t)((const uint16_t *)d.table)[y];
  if (d.mode == XD_POPCOUNT) return (uint32_t)__popcll(y);
  uint32_t idx = 0;
  for (int t = 0; t < d.nterms; t++) idx |= (uint32_t)(__popcll(y & d.masks[t]) & 1) << t;
  return idx;
}
// Diagonal entry of basis state y from a set's table: lut[index] (L = table length), or for
// XD_QUBIT the product of the four 256-entry factor tables over the 8-bit slices of y.
template <typename T2>
__device__ __forceinline__ T2 xdiag_value(const XDiag &d, const T2 *lut, uint64_t y, uint64_t N) {
  if (d.mode != XD_QUBIT) return lut[xdiag_index(d, y)];
  T2 D = lut[y & 255];
  for (int h = 1; h < 4; h++) {
    if (N <= (1ull << (8 * h))) break;
    const T2 f = lut[256 * h + ((y >> (8 * h)) & 255)];
    const T2 o{D.x * f.x - D.y * f.y, D.x * f.y + D.y * f.x};
    D = o;
  }
  return D;
}
unsigned xdiag_blocks(uint64_t N);
int xwht_passes(int n, int precision);
hipError_t launch_xlut(int precision, const double *vals, int len, const double *angles, int stride, int off,
                       double sign, int nsets, void *out, hipStream_t s);
hipError_t launch_xlut_q(int precision, int n, const double *angles, int stride, int off, double sign, int nsets,
                         void *out, hipStream_t s);
hipError_t launch_xdiag(int precision, int nv, int gsums, void *phi, void *lam, uint64_t N, const XDiag &d,
                        const void *luts, int lut_len, const double *gv, double gshift, double *partials,
                        int nsets, hipStream_t s);
hipError_t launch_xend(int precision, const void *phi, void *lam, uint64_t N, const XDiag &d, const double *vals,
                       int lut_len, double c0, double *partials, int nsets, hipStream_t s);
hipError_t launch_xfill(int precision, void *v, uint64_t total, double u0, hipStream_t s);
hipError_t launch_xfinal(const double *partials, int nblk, int nsums, int nsets, double *out, int ostride, int ooff,
                         hipStream_t s);
hipError_t launch_xwht(int precision, int nv, void *phi, void *lam, int n, int nsets, hipStream_t s);
// Walsh-Hadamard transform with register tiles of 2^13 (complex64) or 2^12 (complex128)
// amplitudes, for n >= wht_min_bits(precision).
hipError_t launch_wht_tiles(int precision, int nv, void *phi, void *lam, int n, int nsets, hipStream_t s,
                            const XDiag *pre = nullptr, const void *luts = nullptr, int lut_len = 0);
// W applied to one vector after multiplying it by a diagonal (forward steps of the X-product
// path); the multiply is fused into the first transform pass when the register tiles apply.
hipError_t launch_xwht_pre(int precision, void *phi, int n, int nsets, const XDiag &d, const void *luts, int lut_len,
                           hipStream_t s);
int wht_tile_passes(int n, int precision);
int wht_min_bits(int precision);

// Whole-state evaluation with the state in registers, for n = 12, 13 (FP32) or n = 12 (FP64):
// every item must have that n and table width.
bool whole_supported(int precision, int n);
hipError_t launch_whole(int precision, int n, int tbytes, const SmallItem *items, int n_items, int max_lut,
                        const double *angles, int p, int grad, double *out, hipStream_t s, int stage = 0);
hipError_t launch_scale_copy(int precision, const void *src, void *dst, uint64_t N, double re,
                             double im, uint64_t flip, hipStream_t s);
size_t pass_lds_bytes(int precision, int tbytes, int lut_len);
// Split-FP16 MFMA product (qaoa_gemm.hip): C[m + n ldc] = sum_k M[m][k] S[n][k] for m < M,
// n < cols, every operand given as FP16 hi and 2^11-scaled lo planes. The state planes (S) are
// rows of kp halves (kp a multiple of SPLIT_KQUANT) in the blocked layout of
// split_plane_offset, roundup(cols, SPLIT_TILE) rows, zero-padded; the matrix planes (M) are in
// the fragment-major layout of split_frag_offset, roundup(M, SPLIT_MTILE) rows of kp halves,
// zero-padded.
constexpr int SPLIT_TILE = 128, SPLIT_KTILE = 32;
constexpr int SPLIT_MTILE = 256;   // rows of C per workgroup
constexpr int SPLIT_KQUANT = 128;  // K of four LDS stages: the padded K of every plane is a multiple
// Offset (in halves) of element (row r, k) of a blocked plane: blocks of SPLIT_TILE rows x
// SPLIT_KTILE halves, one per (row tile, K tile), K tiles of a row tile consecutive; inside a
// block row rr holds its four 16-byte chunks in the order c ^ ((rr >> 2) & 3).
__host__ __device__ inline int64_t split_plane_offset(int64_t r, int64_t k, int64_t kp) {
  const int64_t rt = r / SPLIT_TILE, kt = k / SPLIT_KTILE, rr = r % SPLIT_TILE, kk = k % SPLIT_KTILE;
  return (rt * (kp / SPLIT_KTILE) + kt) * (SPLIT_TILE * SPLIT_KTILE) + rr * SPLIT_KTILE +
         8 * ((kk >> 3) ^ ((rr >> 2) & 3)) + (kk & 7);
}
// Offset (in halves) of element (row r, k) of a fragment-major plane: one 1 KB chunk per (block
// of 32 rows, K step of 16), K steps of a row block consecutive; inside a chunk, lane l of a
// wave holds the 16 bytes of row (l % 32), k = 8 (l / 32) .. + 7 of the step (the operand
// fragment of the 32 x 32 x 16 MFMA), so one wave reads a fragment with one contiguous 1 KB load.
__host__ __device__ inline int64_t split_frag_offset(int64_t r, int64_t k, int64_t kp) {
  const int64_t rb = r >> 5, ks = k >> 4, lane = (r & 31) + 32 * ((k >> 3) & 1);
  return ((rb * (kp >> 4) + ks) * 64 + lane) * 8 + (k & 7);
}
// Write the complex value (re, im) of row x of angle set s as the next split product's input:
// FP16 hi and 2^11-scaled lo of the real part (state column 2s) and the imaginary part (column
// 2s + 1), into the blocked planes lo = B, hi = B + plane (rows of ldb halves).
__device__ __forceinline__ void split_emit(_Float16 *B, int64_t ldb, int64_t plane, int64_t x, int s, float re,
                                           float im) {
  const _Float16 hr = (_Float16)re, hi = (_Float16)im;
  const int64_t c0 = split_plane_offset(2 * s, x, ldb), c1 = split_plane_offset(2 * s + 1, x, ldb);
  B[plane + c0] = hr;
  B[c0] = (_Float16)((re - (float)hr) * 2048.0f);
  B[plane + c1] = hi;
  B[c1] = (_Float16)((im - (float)hi) * 2048.0f);
}
// Epilogues fused into the split product (the elementwise steps of the eigenbasis mixers,
// applied to the product's tile while it is in registers). Rows are rows of the product
// (eigen-index r after V^T, state index x after V), column pairs (2s, 2s + 1) angle set s.
enum {
  SE_PLAIN = 0,   // C[m + n ldc] = product
  SE_EIG = 1,     // t *= e^{-i beta_s D_r}; ck <- t (if ck); emit t
  SE_PHASE = 2,   // psi *= lut_s[C(x)]; ck <- psi (if ck); emit psi
  SE_LAST = 3,    // C <- psi; part0 += |psi|^2 C(x), part1 += |psi|^2; emit (C(x) - c0) psi if bout
  SE_REIG = 4,    // part0 += D_r Im(conj(t) ckr); t *= e^{+i beta_s D_r}; emit t
  SE_RPHASE = 5,  // part0 += (C(x) - c0) Im(conj(lam) ckr); lam *= lut_s[C(x)]; emit lam if bout
};
struct SplitEpi {
  float *C;                  // SE_PLAIN, SE_LAST: FP32 output, column-major, ld ldc
  int64_t ldc;
  _Float16 *bout;            // next product's input planes (lo at bout, hi at bout + bplane)
  int64_t bld, bplane;
  float *ck;                 // SE_EIG, SE_PHASE: kept copy (column-major, ld ldc), may be null
  const float *ckr;          // SE_REIG, SE_RPHASE: the forward sweep's kept copy
  const double *D;           // eigenvalues
  const double *betas;       // beta of each set
  const void *table;         // cost table index per state (tbytes 1 or 2)
  int tbytes;
  const double *vals;        // cost value of each table index
  double c0;
  const float2 *luts;        // lut_len entries per set
  int lut_len;
  double *part0, *part1;     // partial sums [s * nblk + row tile]
  int nblk;
  float *ws;                 // split_gemm_ws_bytes of workspace when that is nonzero
};
hipError_t launch_split_gemm_epi(int mode, const void *st_h, const void *st_l, const void *m_h, const void *m_l,
                                 int64_t kp, int M, int cols, const SplitEpi &e, hipStream_t s);
// Workspace (bytes) of one product of M rows, cols columns and padded depth kp: nonzero when the
// product runs the XCD-balanced schedule, whose K-split tiles keep their partial sums there.
size_t split_gemm_ws_bytes(int M, int cols, int64_t kp);
// dst <- src, bytes a multiple of 16, both 16-byte aligned (the HBM copy roof).
hipError_t launch_stream_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
// Grover path (qaoa_grover.hip)
hipError_t launch_hist_table(const void *table, int tbytes, uint64_t N, int nbins, unsigned long long *counts,
                             hipStream_t s);
size_t enum_full_lds(int nbins, bool priv);
// masks == nullptr: adjacency-list walk; else nw (1, 2, 4 or 8) neighbour masks per vertex, one
// per distinct edge weight wvals[j] (padding classes: empty mask, weight 0), and their popcounts
// mdeg
hipError_t launch_enum_full(int n, int m, const int32_t *eu, const int32_t *ev, const int32_t *ew,
                            const int32_t *adj_off, const int32_t *adj, const uint64_t *masks, const int32_t *mdeg,
                            const int32_t *wvals, int nw, int lo, uint64_t base, uint64_t nthreads, int nbins,
                            bool priv, unsigned long long *counts, hipStream_t s);
hipError_t launch_enum_hw(int n, int k, int m, const int32_t *eu, const int32_t *ev, const int32_t *ew,
                          const int64_t *binom, uint64_t r0, uint64_t per, uint64_t total, uint64_t nthreads,
                          int nbins, unsigned long long *counts, hipStream_t s);
hipError_t launch_grover(const GroverItem *items, int n_items, const double *angles, int p, int grad, double *out,
                         hipStream_t s);
hipError_t launch_grover_expand(const void *table, int tbytes, uint64_t N, const double2 *amp, void *out,
                                int precision, hipStream_t s);

}  // namespace qaoa
