// Internal interface between the host runtime (nmf_runtime.hip) and the
// gfx950 kernels (nmf_kernels.hip).  Each launcher enqueues one kernel on
// `st` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmfk {

// Supported padded ranks: the rank dimension of every internal buffer is
// padded with zeros to one of these.
inline int padded_rank(int r) {
  if (r <= 16) return 16;
  if (r <= 32) return 32;
  if (r <= 64) return 64;
  if (r <= 128) return 128;
  return 256;
}

// Tile shape of the "NT" product  C[m][c] = sum_k X[m][k] * Y[c][k]
// (both operands contiguous along k).  BM x BN output tile per workgroup.
struct NtCfg {
  int id;      // template instance
  int bm, bn;  // tile
  int threads;
  int bk;       // reduction slots per LDS stage (float32)
  int bk_bf16;  // reduction slots per LDS stage (bf16)
};
// Tile shape of the "TN" product  C[m][c] = sum_k A[k][m] * B[k][c]
// (both operands contiguous along the output dimension, k the row index).
struct TnCfg {
  int id;
  int bm, bn;
  int threads;
  int bk;
};

// Gram reduction carried by a product kernel (see gram_reduce_slice):
// G[e] = sum_{q < count} part[q * elems + e] for e < elems.  part == nullptr
// disables it.
struct GramRed {
  const float* part;
  int count;
  int elems;
  float* G;
  int at_end;  // V-streaming products: reduce after the main loop, not before
  int wide;    // chunks of 32 elements per workgroup (large Grams), else one element per 32 lanes
};

NtCfg nt_config(int rp, bool gram);
NtCfg nt_config_by_id(int id);
TnCfg tn_config_by_id(int id);
int nt_config_count();
int tn_config_count();
TnCfg tn_config(int rp, bool gram);
NtCfg nt_bf16_config(int rp, bool gram);

// ---- FP32 products with split-K partials --------------------------------
// part[s][m][c] (row pitch ldp, split pitch sp) for m < round_up(M, bm),
// c < round_up(N, bn).  Rows m >= M / k >= K read as zero.
hipError_t launch_gemm_nt(const NtCfg& cfg, const float* X, int64_t ldx,
                          int64_t M, const float* Y, int64_t ldy, int64_t N,
                          int64_t K, int splits, int64_t kchunk, float* part,
                          int64_t ldp, int64_t sp, const GramRed& gr,
                          hipStream_t st);
hipError_t launch_gemm_tn(const TnCfg& cfg, const float* A, int64_t lda,
                          int64_t M, const float* B, int64_t ldb, int64_t N,
                          int64_t K, int splits, int64_t kchunk, float* part,
                          int64_t ldp, int64_t sp, const GramRed& gr,
                          hipStream_t st);

// ---- V-streaming NT product through an asynchronous LDS ring ------------
// part[s][m][c] = sum_k X[m][k] Y[c][k], float32 or bf16 operands (float32
// accumulation).  X and Y rows must be readable up to round_up(M, bm) and
// round_up(N, bn) and along k up to K, with zeros beyond the data; K and
// kchunk multiples of 256; pitches (in elements) multiples of 64 bytes.
struct DmaCfg {
  int id;
  int bm, bn;
  int threads;
};
// Tile of the V-streaming products for padded rank rp; narrow: the 64-wide
// tiles for problems whose default tiling leaves fewer than 256 workgroups;
// bf16: the tile for the BF16 tier's products.
DmaCfg dma_config(int rp, bool pass1, bool narrow = false, bool bf16 = false);
DmaCfg dma_config_by_id(int id);
hipError_t launch_nt_dma(const DmaCfg& cfg, bool bf16, const void* X, int64_t ldx,
                         int64_t M, const void* Y, int64_t ldy, int64_t N, int64_t K,
                         int splits, int64_t kchunk, float* part, int64_t ldp,
                         int64_t sp, const GramRed& gr, hipStream_t st);

// ---- BF16 NT product (16x16x32 MFMA, FP32 accumulation) ------------------
hipError_t launch_gemm_nt_bf16(const NtCfg& cfg, const uint16_t* X,
                               int64_t ldx, int64_t M, const uint16_t* Y,
                               int64_t ldy, int64_t N, int64_t K, int splits,
                               int64_t kchunk, float* part, int64_t ldp,
                               int64_t sp, const GramRed& gr, hipStream_t st);

// G[m][c] = sum_s part[s][m][c] for m, c < rp; written with pitch rp.
// With bf16 != nullptr also writes the bfloat16 rounding of G there.
hipError_t launch_reduce_gram(const float* part, int64_t ldp, int64_t sp,
                              int splits, int rp, float* G, uint16_t* Gbf,
                              hipStream_t st);

// Block shapes of the update kernels: rank entries per thread of the W
// update (4 or 1) and columns per block of the H update (64, 32 or 16),
// narrowed when the full shape would leave fewer than 256 workgroups.
int update_w_kpt(int rp, int64_t p);
int update_h_cols(int64_t n);
// Number of workgroups of the update kernels (grid-stride; capped at cap).
int update_grid(int rp, int64_t p, int cap, int kpt);
int update_h_grid(int64_t n, int cap, int cols);

// W half-step epilogue.  Wp (ppad x rp) holds the current W; A partials are
// part[s][i][k] (pitch ldp, split pitch sp).  Writes the new W to Wp, to the
// caller's W (p x r) and, when given, to WT (float32) or WbT (bf16), both
// transposed (rp x ldwt).
// gout != nullptr (rp <= 64): also writes per-workgroup Grams of the new W
// (grid x rp x rp).  gram_only: no update, Grams of the current W only.
hipError_t launch_update_w(int rp, int64_t p, int r, const float* part,
                           int64_t ldp, int64_t sp, int splits, const float* G,
                           float* Wp, float* Wcaller, float* WT, uint16_t* WbT,
                           int64_t ldwt, bool bf16, float* gout, int grid,
                           int kpt, bool gram_only, hipStream_t st);

// H half-step epilogue.  Hp (rp x ldh) holds the current H; S partials are
// part[s][k][j].  Writes Hp, the caller's H (r x n) and, for the BF16 tier,
// Hb (rp x ldh); gout/gram_only as for the W update (Grams of H H^T).
hipError_t launch_update_h(int rp, int64_t n, int r, const float* part,
                           int64_t ldp, int64_t sp, int splits, const float* G,
                           float* Hp, int64_t ldh, float* Hcaller, uint16_t* Hb,
                           bool bf16, float* gout, int grid, int cols,
                           bool gram_only, hipStream_t st);

// launch_update_h for rp <= 64 with the denominator G H and the Gram
// partials on the matrix cores (gram_only: the Gram partials of H alone;
// early_g: G is loaded together with the first block's other loads, for
// grids of at most one workgroup per CU, where the registers that costs do
// not cut the workgroups that run at once).
hipError_t launch_update_h_mf(int rp, int64_t n, int r, const float* part, int64_t ldp,
                              int64_t sp, int splits, const float* G, float* Hp, int64_t ldh,
                              float* Hcaller, uint16_t* Hb, bool bf16, float* gout, int grid,
                              int cols, bool gram_only, bool early_g, hipStream_t st);

// Objective partials: one double per 64 x 64 tile of V - W H.
hipError_t launch_objective(int rp, const float* V, int64_t ldv, int64_t p,
                            int64_t n, const float* Wp, const float* Hp,
                            int64_t ldh, double* part, hipStream_t st);
// The same partials with W H formed on the float64 matrix cores (the same
// tiles and order of tile sums; the k order inside a dot product differs).
hipError_t launch_objective_mma(int rp, const float* V, int64_t ldv, int64_t p,
                                int64_t n, const float* Wp, const float* Hp,
                                int64_t ldh, double* part, hipStream_t st);
int64_t objective_parts(int64_t p, int64_t n);
// out[0] = sum of part[0..count) in a fixed order.
hipError_t launch_reduce_f64(const double* part, int64_t count, double* out,
                             hipStream_t st);

// Elementwise helpers.
hipError_t launch_copy_pad(const float* src, int64_t lds, int64_t rows,
                           int64_t cols, float* dst, int64_t ldd,
                           hipStream_t st);  // dst[i][j] = src[i][j]
hipError_t launch_fill_f32(float* dst, int64_t count, float v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* dst, int64_t count, uint32_t v,
                           hipStream_t st);
// bf16 copy (RNE) of src (rows x cols) into dst with pitch ldd; with
// transpose, dst[j][i] = bf16(src[i][j]).
hipError_t launch_cast_bf16(const float* src, int64_t lds, int64_t rows,
                            int64_t cols, uint16_t* dst, int64_t ldd,
                            bool transpose, hipStream_t st);
// dst[j][i] = src[i][j] (float32), pitch ldd.
hipError_t launch_transpose_f32(const float* src, int64_t lds, int64_t rows,
                                int64_t cols, float* dst, int64_t ldd,
                                hipStream_t st);
// Scale every nonzero column of W (p x r) to unit norm and the matching row
// of H (r x n) by that norm; norms: r floats of scratch.
hipError_t launch_gauge(float* W, int64_t p, int r, float* H, int64_t n, float* norms,
                        hipStream_t st);
// Least-squares warm-start dictionary (rp <= 64): W = max(A (G + delta I)^-1,
// floor) from the pass-1 partials A (part, split layout as for the W update)
// and G = G_H; delta = 1e-6 tr(G)/r, floor = floor_rel * max(W).  Writes Wp
// (pitch rp) and the caller's W (p x r).  ginv: rp * rp doubles of scratch,
// maxbits: one word.
hipError_t launch_ls_refit(const float* G, int rp, int r, int64_t p, const float* part,
                           int64_t ldp, int64_t sp, int splits, double* ginv,
                           uint32_t* maxbits, float floor_rel, float* Wp, float* Wcaller,
                           hipStream_t st);
// ---- Poisson (KL) multiplicative update (padded ranks 16, 32, 64) --------
// Tiles of the two numerator passes: pass 1 bm1 x bn1 (data rows x ranks),
// pass 2 bm2 x bn2 (ranks x data columns); every tile holds all rp ranks.
void kl_tiles(int rp, int* bm1, int* bn1, int* bm2, int* bn2);
// part[s][m][c] = sum_k X'[m][k] Y'[c][k] with the data operand (pass 1: X =
// V, pass 2: Y = V^T) replaced by V / (W H) (zero where V is zero); G is the
// factor not streamed: pass 1 W (ppad x rp, ldg = rp), pass 2 H (rp x ldg).
hipError_t launch_kl_pass(int rp, bool pass1, const float* X, int64_t ldx, int64_t M,
                          const float* Y, int64_t ldy, int64_t N, int64_t K, int splits,
                          int64_t kchunk, const float* G, int64_t ldg, float* part,
                          int64_t ldp, int64_t sp, hipStream_t st);
// den[k] = sum_{j<n} H[k][j], den[rp + k] = sum_{i<p} W[i][k] (float64 sums).
hipError_t launch_kl_sums(const float* Wp, int rp, int64_t p, const float* Hp, int64_t ldh,
                          int64_t n, float* den, hipStream_t st);
// The square-root updates of W and H from the pass partials and den.
hipError_t launch_kl_update_w(const float* part, int64_t ldp, int64_t sp, int splits,
                              const float* den, float* Wp, int rp, int64_t p, int r, float* WT,
                              int64_t ldwt, float* Wc, hipStream_t st);
hipError_t launch_kl_update_h(const float* part, int64_t ldp, int64_t sp, int splits,
                              const float* den, float* Hp, int64_t ldh, int rp, int64_t n,
                              int r, float* Hc, hipStream_t st);
// Poisson objective partials, one double per 64 x 64 tile (grid as
// launch_objective): sum [v ln b - b], b = W H in float64, 0 ln 0 = 0.
hipError_t launch_kl_objective(int rp, const float* V, int64_t ldv, int64_t p, int64_t n,
                               const float* Wp, const float* Hp, int64_t ldh, double* part,
                               hipStream_t st);

// ---- QN(q) acceleration of the multiplicative map (x = [Wp | Hp]) --------
int qn_max_q();      // largest q the kernels hold
int qn_dot_blocks();  // rows of the dot-product partials (dpart: blocks x 3 q)
// dst = src (D floats, D % 4 == 0).
hipError_t launch_qn_copy(const float* src, float* dst, int64_t D, hipStream_t st);
// Ring slot s = state[0] % q of U, V (float64, q x D): u = x1 - x0, v = x2 - x1.
hipError_t launch_qn_pairs(const float* x0, const float* x1, const float* x2, double* U,
                           double* V, int64_t D, int q, const int32_t* state, hipStream_t st);
// Slot s's row / column of U^T U and U^T V (GUU, GUV: q_max x q_max), then
// coef = (U^T U - U^T V)^-1 U^T u_s over the filled slots; state[2] = regular.
hipError_t launch_qn_dots_solve(const double* U, const double* V, int64_t D, int q,
                                int32_t* state, double* dpart, double* GUU, double* GUV,
                                double* coef, hipStream_t st);
// xq = max(x1 + V coef, kappa x1) (x1 if singular); state[3] |= infeasible.
hipError_t launch_qn_combine(const float* x1, const double* V, const double* coef, int64_t D,
                             int q, float kappa, int32_t* state, float* xq, hipStream_t st);
// take = regular && feasible && fvals[1] <= fvals[0]; fout[state[0]] = the
// accepted objective; state[0]++, state[1] += take.
hipError_t launch_qn_select(const double* fvals, int32_t* state, double* fout, int32_t cap,
                            hipStream_t st);
// If taken: [Wp | Hp] = xq and its derived copies (caller's W and H; W^T in
// float32, or bf16(W^T) and bf16(H)); pointers not used by the tier are null.
hipError_t launch_qn_commit(const int32_t* state, const float* xq, float* Wp, int64_t ppad, int rp,
                            int64_t npad, int64_t p, int r, int64_t n, float* Wc, float* Hc,
                            float* WT, uint16_t* WbT, int64_t ldwt, uint16_t* Hb, hipStream_t st);

// flag |= 1 if some V entry is negative or non-finite.
hipError_t launch_validate(const float* V, int64_t ldv, int64_t p, int64_t n,
                           uint32_t* flag, hipStream_t st);
// dst[i][j] = U(0,1) from Philox4x32-10(key = seed, counter = (i*cols + j,
// stream_id, 0, 0)) for i < rows, j < cols; pitch ldd.
hipError_t launch_uniform(float* dst, int64_t rows, int64_t cols, int64_t ldd,
                          uint64_t seed, uint32_t stream_id, hipStream_t st);

}  // namespace nmfk
