// Host runtime behind the C ABI of include/nmf.h: argument checks, device
// workspace, tile/split selection and the per-iteration launch sequence of
// Algorithm 1 (NNMF):
//
//   W half-step:  A = V H^T (split-K partials)  ->  W <- W * A / (W G_H)
//                 -> G_W = W^T W                     (for the H half-step)
//   H half-step:  S = W^T V (split-K partials)  ->  H <- H * S / (G_W H)
//                 -> G_H = H H^T                     (for the next W half-step)
//
// Internal layout (row-major, zero padded; ppad = round_up(p, 256),
// npad = round_up(n, 256), rp = padded rank; the streamed copies get row
// pitches from spread_pitch, i.e. npad / ppad plus a pad of 128 to 512 bytes
// when that is a multiple of 4 KB):
//   Wp (ppad x rp), Hp (rp x npad), G_H and G_W (rp x rp)
//   FP32:  V itself when p, n are multiples of 256 and its pitch is not a
//          multiple of 4 KB (else a padded ppad x npad copy),
//          VT = V^T (npad x ppad), WT = W^T (rp x ppad)
//   BF16:  Vb = bf16(V) (ppad x npad), VTb = bf16(V^T) (npad x ppad),
//          Hb = bf16(H) (rp x npad), WbT = bf16(W^T) (rp x ppad)
// Both V-streaming products are NT products through the LDS copy ring:
//   pass 1  A = V H^T   X = V / Vb,   Y = Hp / Hb,  K = npad
//   pass 2  S = W^T V   X = WT / WbT, Y = VT / VTb, K = ppad
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/nmf.h"
#include "nmf_internal.h"

using namespace nmfk;

namespace {

constexpr int64_t kMaxDim = 4000000;  // objective grid.y = ceil(p / 64) <= 65535
constexpr int kGraphLevels = 5;        // graphs of 1, 2, 4, 8 and 16 iterations

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Row pitch for a matrix streamed through the copy ring: a pitch that is a
// multiple of 4 KB puts the 100+ rows of one ring stage on the same few HBM
// channels, so such pitches get pad_bytes more.  Measured at 4096 x 16384,
// rank 16, FP32 (pass 1 on V, pass 2 on V^T, microseconds per launch):
// pad 0: 84 / 69; 128 B: 52 / 74; 256 B: 53 / 50; 512 B: 80 / 50;
// 1 KB: 53 / 50.  The BF16 copies are insensitive (128 B is marginally best).
inline int64_t spread_pitch(int64_t elems, int esize, int64_t pad_bytes) {
  return (elems * esize) % 4096 == 0 ? elems + pad_bytes / esize : elems;
}

int64_t env_int(const char* name, int64_t dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  const long long x = std::strtoll(v, &end, 10);
  return (end && *end == 0 && x >= 0) ? (int64_t)x : dflt;
}

struct Split {
  int splits = 1;
  int64_t kchunk = 0;
  int64_t ldp = 0;   // partial row pitch
  int64_t rows = 0;  // partial rows
  int64_t sp = 0;    // split pitch
};

// Split the reduction dimension K so that the grid has about `target`
// workgroups while every split keeps at least `min_steps` stages of `bk`.
Split plan_split(int64_t M, int64_t N, int64_t K, int bm, int bn, int bk, int64_t target,
                 int64_t min_steps) {
  Split s;
  const int64_t tiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  const int64_t steps = (K + bk - 1) / bk;
  int64_t want = std::max<int64_t>(1, target / std::max<int64_t>(1, tiles));
  want = std::min<int64_t>(want, std::max<int64_t>(1, steps / min_steps));
  want = std::min<int64_t>(want, 64);
  const int64_t per = (steps + want - 1) / want;
  s.kchunk = per * bk;
  s.splits = (int)((K + s.kchunk - 1) / s.kchunk);
  if (s.splits < 1) s.splits = 1;
  s.rows = round_up(M, bm);
  s.ldp = round_up(N, bn);
  s.sp = s.rows * s.ldp;
  return s;
}

}  // namespace

struct nmf_ctx {
  int device = 0;
  int cus = 0;  // compute units of the device
  hipStream_t st = nullptr;
  int64_t p = 0, n = 0, ldv = 0;
  int r = 0, rp = 0;
  nmf_options opt{};
  const float* Vuser = nullptr;
  float* Wuser = nullptr;
  float* Huser = nullptr;

  const float* Vk = nullptr;  // V as read by the kernels
  int64_t ldvk = 0;
  int64_t ppad = 0, npad = 0;
  // row pitches (elements) of the streamed copies: bf16(V), V^T / bf16(V^T)
  // and W^T / bf16(W^T); see spread_pitch
  int64_t lvb = 0, lvt = 0, lwt = 0;

  // workspace (one allocation, carved)
  void* ws = nullptr;
  float* Vcopy = nullptr;
  float* Wp = nullptr;
  float* Hp = nullptr;
  float* GH = nullptr;
  float* GW = nullptr;
  float* part1 = nullptr;
  float* part2 = nullptr;
  float* partg = nullptr;
  float* gpw = nullptr;  // per-workgroup Grams of W from the W update (fused path)
  float* gph = nullptr;  // per-workgroup Grams of H from the H update (fused path)
  double* fpart = nullptr;
  uint32_t* flag = nullptr;   // [0] validation, [1] refit maximum
  double* lsinv = nullptr;    // (G_H + delta I)^-1 for nmf_refit_w
  float* VT = nullptr;
  float* WT = nullptr;
  uint16_t* Vb = nullptr;
  uint16_t* VTb = nullptr;
  uint16_t* Hb = nullptr;
  uint16_t* WbT = nullptr;
  double* hostbuf = nullptr;  // pinned, coherent, 4 doubles: [0] reads, [2..3] checks
  double* hostbuf_dev = nullptr;  // the same memory as the device addresses it
  hipEvent_t chk_ev[2] = {nullptr, nullptr};  // solve: check values written

  bool bf16 = false;
  bool kl = false;        // Poisson (KL) square-root update instead of Euclidean
  float* kl_den = nullptr;  // Poisson: 2 x rp denominators (row sums of H, column sums of W)
  bool fuse = false;      // rp <= 64: Grams formed in the update kernels
  int gram_at_end = 0;    // the products reduce the Gram partials after their loop
  int gram_wide = 0;      // ... in chunks of 32 elements per workgroup
  int uw_grid = 1, uh_grid = 1;
  int uw_kpt = 4, uh_cols = 64;  // block shapes of the update kernels
  DmaCfg d1{}, d2{};      // the two V-streaming products
  NtCfg cgh{};            // separate Gram products (rp > 64)
  TnCfg cgw{};
  Split s1, s2, sgh, sgw;
  int64_t nparts = 0;
  double nv2 = 0.0;  // ||V||_F^2 in float64

  // captured iterations (use_graph): graph j runs 2^j iterations
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gp[kGraphLevels] = {};

  // QN(q) acceleration (allocated by the first nmf_solve_qn)
  int qn_q = 0;
  void* qn_ws = nullptr;
  float *qx0 = nullptr, *qx1 = nullptr, *qxq = nullptr;
  double *qU = nullptr, *qV = nullptr, *qdpart = nullptr, *qGUU = nullptr, *qGUV = nullptr;
  double *qcoef = nullptr, *qf = nullptr;
  int32_t* qst = nullptr;
  double* qfout = nullptr;      // pinned, coherent: accepted objective per QN iteration
  double* qfout_dev = nullptr;  // the same memory as the device addresses it
  hipGraphExec_t qn_graph = nullptr;

  // stage profiler (HIP events on st)
  bool prof = false;
  int32_t prof_cap = 0;
  std::vector<hipEvent_t> ev;   // 2 per record
  std::vector<int> ev_stage;    // stage per record
  int32_t prof_used = 0;
};

#define TRY_HIP(expr)                      \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return NMF_EDEVICE; \
  } while (0)
#define TRY(expr)                       \
  do {                                  \
    nmf_status s_ = (expr);             \
    if (s_ != NMF_OK) return s_;        \
  } while (0)

namespace {

// Brackets one stage with profiler events when profiling is on.
struct StageTimer {
  nmf_ctx* c;
  int rec = -1;
  StageTimer(nmf_ctx* ctx, int stage) : c(ctx) {
    if (c->prof && c->prof_used < c->prof_cap) {
      rec = c->prof_used++;
      c->ev_stage[rec] = stage;
      if (hipEventRecord(c->ev[2 * rec], c->st) != hipSuccess) rec = -1;
    }
  }
  ~StageTimer() {
    if (rec >= 0) (void)hipEventRecord(c->ev[2 * rec + 1], c->st);
  }
};

void profile_release(nmf_ctx* c) {
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_stage.clear();
  c->prof = false;
  c->prof_cap = 0;
  c->prof_used = 0;
}

const GramRed kNoGram = {nullptr, 0, 0, nullptr, 0, 0};

nmf_status check_ptr(const void* p) {
  if (!p) return NMF_EINVAL;
  if (reinterpret_cast<uintptr_t>(p) % 4 != 0) return NMF_EINVAL;
  return NMF_OK;
}

// Gram G_H = Hp Hp^T (or its bf16 analogue) from the current H.
nmf_status gram_h(nmf_ctx* c) {
  StageTimer t(c, NMF_STAGE_GRAM_H);
  if (c->bf16) {
    TRY_HIP(launch_gemm_nt_bf16(c->cgh, c->Hb, c->npad, c->rp, c->Hb, c->npad, c->rp, c->n,
                                c->sgh.splits, c->sgh.kchunk, c->partg, c->sgh.ldp, c->sgh.sp,
                                kNoGram, c->st));
  } else {
    TRY_HIP(launch_gemm_nt(c->cgh, c->Hp, c->npad, c->rp, c->Hp, c->npad, c->rp, c->n,
                           c->sgh.splits, c->sgh.kchunk, c->partg, c->sgh.ldp, c->sgh.sp, kNoGram,
                           c->st));
  }
  TRY_HIP(launch_reduce_gram(c->partg, c->sgh.ldp, c->sgh.sp, c->sgh.splits, c->rp, c->GH, nullptr,
                             c->st));
  return NMF_OK;
}

// Gram G_W = Wp^T Wp (or its bf16 analogue) from the current W.
nmf_status gram_w(nmf_ctx* c) {
  StageTimer t(c, NMF_STAGE_GRAM_W);
  if (c->bf16) {
    TRY_HIP(launch_gemm_nt_bf16(c->cgh, c->WbT, c->lwt, c->rp, c->WbT, c->lwt, c->rp, c->p,
                                c->sgw.splits, c->sgw.kchunk, c->partg, c->sgw.ldp, c->sgw.sp,
                                kNoGram, c->st));
  } else {
    TRY_HIP(launch_gemm_tn(c->cgw, c->Wp, c->rp, c->rp, c->Wp, c->rp, c->rp, c->p, c->sgw.splits,
                           c->sgw.kchunk, c->partg, c->sgw.ldp, c->sgw.sp, kNoGram, c->st));
  }
  TRY_HIP(launch_reduce_gram(c->partg, c->sgw.ldp, c->sgw.sp, c->sgw.splits, c->rp, c->GW, nullptr,
                             c->st));
  return NMF_OK;
}

nmf_status half_w(nmf_ctx* c) {
  // G_H: reduced inside the product from the H update's per-workgroup Grams
  const GramRed gr =
      c->fuse ? GramRed{c->gph, c->uh_grid, c->rp * c->rp, c->GH, c->gram_at_end, c->gram_wide}
              : kNoGram;
  {
    StageTimer t(c, NMF_STAGE_GEMM_VHT);
    const void* X = c->bf16 ? static_cast<const void*>(c->Vb) : static_cast<const void*>(c->Vk);
    const void* Y = c->bf16 ? static_cast<const void*>(c->Hb) : static_cast<const void*>(c->Hp);
    TRY_HIP(launch_nt_dma(c->d1, c->bf16, X, c->bf16 ? c->lvb : c->ldvk, c->p, Y, c->npad,
                          c->rp, c->npad, c->s1.splits, c->s1.kchunk, c->part1, c->s1.ldp,
                          c->s1.sp, gr, c->st));
  }
  {
    StageTimer t(c, NMF_STAGE_UPDATE_W);
    TRY_HIP(launch_update_w(c->rp, c->p, c->r, c->part1, c->s1.ldp, c->s1.sp, c->s1.splits,
                            c->GH, c->Wp, c->Wuser, c->bf16 ? nullptr : c->WT,
                            c->bf16 ? c->WbT : nullptr, c->lwt, c->bf16,
                            c->fuse ? c->gpw : nullptr, c->uw_grid, c->uw_kpt, false, c->st));
  }
  return c->fuse ? NMF_OK : gram_w(c);
}

hipError_t update_h_call(nmf_ctx* c, const float* part, int64_t ldp, int64_t sp, int splits,
                         const float* G, uint16_t* Hb, float* gout, bool gram_only);

nmf_status half_h(nmf_ctx* c) {
  const GramRed gr =
      c->fuse ? GramRed{c->gpw, c->uw_grid, c->rp * c->rp, c->GW, c->gram_at_end, c->gram_wide}
              : kNoGram;
  {
    StageTimer t(c, NMF_STAGE_GEMM_WTV);
    const void* X = c->bf16 ? static_cast<const void*>(c->WbT) : static_cast<const void*>(c->WT);
    const void* Y = c->bf16 ? static_cast<const void*>(c->VTb) : static_cast<const void*>(c->VT);
    TRY_HIP(launch_nt_dma(c->d2, c->bf16, X, c->lwt, c->rp, Y, c->lvt, c->n, c->ppad,
                          c->s2.splits, c->s2.kchunk, c->part2, c->s2.ldp, c->s2.sp, gr, c->st));
  }
  {
    StageTimer t(c, NMF_STAGE_UPDATE_H);
    TRY_HIP(update_h_call(c, c->part2, c->s2.ldp, c->s2.sp, c->s2.splits, c->GW,
                          c->bf16 ? c->Hb : nullptr, c->fuse ? c->gph : nullptr, false));
  }
  return c->fuse ? NMF_OK : gram_h(c);
}

// One iteration of the Poisson update (both factors from the same iterate):
// the two denominators, the two numerator passes over V and V^T (each
// recomputing its B = W H values on the matrix cores), then the square-root
// updates of W and H.  The denominator kernel is timed as the W Gram stage.
nmf_status kl_iter(nmf_ctx* c) {
  {
    StageTimer t(c, NMF_STAGE_GRAM_W);
    TRY_HIP(launch_kl_sums(c->Wp, c->rp, c->p, c->Hp, c->npad, c->n, c->kl_den, c->st));
  }
  {
    StageTimer t(c, NMF_STAGE_GEMM_VHT);
    TRY_HIP(launch_kl_pass(c->rp, true, c->Vk, c->ldvk, c->p, c->Hp, c->npad, c->rp, c->npad,
                           c->s1.splits, c->s1.kchunk, c->Wp, c->rp, c->part1, c->s1.ldp,
                           c->s1.sp, c->st));
  }
  {
    StageTimer t(c, NMF_STAGE_GEMM_WTV);
    TRY_HIP(launch_kl_pass(c->rp, false, c->WT, c->lwt, c->rp, c->VT, c->lvt, c->n, c->ppad,
                           c->s2.splits, c->s2.kchunk, c->Hp, c->npad, c->part2, c->s2.ldp,
                           c->s2.sp, c->st));
  }
  {
    StageTimer t(c, NMF_STAGE_UPDATE_W);
    TRY_HIP(launch_kl_update_w(c->part1, c->s1.ldp, c->s1.sp, c->s1.splits, c->kl_den, c->Wp,
                               c->rp, c->p, c->r, c->WT, c->lwt, c->Wuser, c->st));
  }
  {
    StageTimer t(c, NMF_STAGE_UPDATE_H);
    TRY_HIP(launch_kl_update_h(c->part2, c->s2.ldp, c->s2.sp, c->s2.splits, c->kl_den, c->Hp,
                               c->npad, c->rp, c->n, c->r, c->Huser, c->st));
  }
  return NMF_OK;
}

// One full iteration of the context's method.
nmf_status iterate(nmf_ctx* c) {
  if (c->kl) return kl_iter(c);
  TRY(half_w(c));
  return half_h(c);
}

// The H update (or, gram_only, the Gram partials of the current H): up to
// rank 64 with its small products on the matrix cores (NMF_UPDATE_H_VALU=1:
// the vector-unit kernel, whose sums run in another order).
hipError_t update_h_call(nmf_ctx* c, const float* part, int64_t ldp, int64_t sp, int splits,
                         const float* G, uint16_t* Hb, float* gout, bool gram_only) {
  static const bool valu = env_int("NMF_UPDATE_H_VALU", 0) != 0;
  if (c->rp <= 64 && !valu)
    return launch_update_h_mf(c->rp, c->n, c->r, part, ldp, sp, splits, G, c->Hp, c->npad,
                              c->Huser, Hb, c->bf16, gout, c->uh_grid, c->uh_cols, gram_only,
                              c->uh_grid <= c->cus, c->st);
  return launch_update_h(c->rp, c->n, c->r, part, ldp, sp, splits, G, c->Hp, c->npad, c->Huser,
                         Hb, c->bf16, gout, c->uh_grid, c->uh_cols, gram_only, c->st);
}

// Euclidean objective partials of (Wp, Hp) into c->fpart: on the float64
// matrix cores from rank 64 up, on the vector units below (where the
// products are few and the matrix-core form's staging dominates: 4096 x
// 16384, rank 16: 116 against 151 us; rank 64: 297 against 265 us; 8192 x
// 32768, rank 256: 3564 against 2703 us).  NMF_OBJECTIVE_VECTOR=1 or =0
// forces one form.
hipError_t euclid_objective(nmf_ctx* c, const float* Wp, const float* Hp, hipStream_t st) {
  static const int64_t force = env_int("NMF_OBJECTIVE_VECTOR", -1);
  // W = 0 (||V||^2, once per context) is a plain streaming sum: the vector
  // kernel's float4 loads do it in half the time
  const bool vec = force >= 0 ? force != 0 : (c->rp < 64 || Wp == nullptr);
  return vec ? launch_objective(c->rp, c->Vk, c->ldvk, c->p, c->n, Wp, Hp, c->npad, c->fpart, st)
             : launch_objective_mma(c->rp, c->Vk, c->ldvk, c->p, c->n, Wp, Hp, c->npad, c->fpart,
                                    st);
}

// Objective partials and their float64 reduction into out (device memory,
// or the mapped pinned host buffer: then no copy operation is needed).
nmf_status objective_async(nmf_ctx* c, const float* Wp, double* out) {
  StageTimer t(c, NMF_STAGE_OBJECTIVE);
  if (c->kl && Wp)
    TRY_HIP(launch_kl_objective(c->rp, c->Vk, c->ldvk, c->p, c->n, Wp, c->Hp, c->npad, c->fpart,
                                c->st));
  else
    TRY_HIP(euclid_objective(c, Wp, c->Hp, c->st));
  TRY_HIP(launch_reduce_f64(c->fpart, c->nparts, out, c->st));
  return NMF_OK;
}

// Objective of the current state (W = Wp, or 0 for Wp == nullptr), written
// by the reduction kernel straight into the pinned host buffer.
nmf_status objective_sync(nmf_ctx* c, const float* Wp, double* f) {
  TRY(objective_async(c, Wp, c->hostbuf_dev));
  TRY_HIP(hipStreamSynchronize(c->st));
  *f = c->hostbuf[0];
  return NMF_OK;
}

void free_ctx(nmf_ctx* c) {
  if (!c) return;
  profile_release(c);
  if (c->qn_graph) (void)hipGraphExecDestroy(c->qn_graph);
  if (c->qn_ws) (void)hipFree(c->qn_ws);
  if (c->qfout) (void)hipHostFree(c->qfout);
  for (hipGraphExec_t g : c->gp)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->ws) (void)hipFree(c->ws);
  if (c->hostbuf) (void)hipHostFree(c->hostbuf);
  for (hipEvent_t e : c->chk_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

// Capture `iters` iterations launched on a private stream into an
// executable graph.  The kernels' arguments are fixed for the context's
// life, so a graph can be replayed on any stream.
nmf_status capture(nmf_ctx* c, int32_t iters, hipGraphExec_t* out) {
  if (!c->cap_stream) TRY_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t user = c->st;
  c->st = c->cap_stream;
  hipGraph_t graph = nullptr;
  nmf_status s = NMF_OK;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->st = user;
    return NMF_EDEVICE;
  }
  for (int32_t it = 0; it < iters && s == NMF_OK; ++it) s = iterate(c);
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  c->st = user;
  if (s != NMF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess || !graph) return NMF_EDEVICE;
  const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return NMF_EDEVICE;
  // upload now, so that the first launch costs what every later one does
  return hipGraphUpload(*out, c->st) == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

constexpr int32_t kQnCap = 65536;  // QN iterations recorded per nmf_solve_qn call
constexpr float kQnKappa = 0.5f;    // projection x >= kappa F(x) of the QN point

int64_t qn_dim(const nmf_ctx* c) { return c->ppad * c->rp + (int64_t)c->rp * c->npad; }

// Enqueue one QN(q) iteration (see nmf_qn.hip): two MM iterations with
// snapshots, the secant pair, the q x q solve, the projected quasi-Newton
// point, both objectives, the device-side choice and its commit, and the
// Grams of the chosen factors for the next MM iteration.
nmf_status qn_enqueue(nmf_ctx* c) {
  const int64_t D = qn_dim(c);
  const int q = c->qn_q;
  TRY_HIP(launch_qn_copy(c->Wp, c->qx0, D, c->st));
  TRY(iterate(c));
  TRY_HIP(launch_qn_copy(c->Wp, c->qx1, D, c->st));
  TRY(iterate(c));
  TRY_HIP(launch_qn_pairs(c->qx0, c->qx1, c->Wp, c->qU, c->qV, D, q, c->qst, c->st));
  TRY_HIP(launch_qn_dots_solve(c->qU, c->qV, D, q, c->qst, c->qdpart, c->qGUU, c->qGUV, c->qcoef,
                               c->st));
  TRY_HIP(launch_qn_combine(c->qx1, c->qV, c->qcoef, D, q, kQnKappa, c->qst, c->qxq, c->st));
  TRY_HIP(euclid_objective(c, c->Wp, c->Hp, c->st));
  TRY_HIP(launch_reduce_f64(c->fpart, c->nparts, c->qf + 0, c->st));
  TRY_HIP(euclid_objective(c, c->qxq, c->qxq + c->ppad * c->rp, c->st));
  TRY_HIP(launch_reduce_f64(c->fpart, c->nparts, c->qf + 1, c->st));
  TRY_HIP(launch_qn_select(c->qf, c->qst, c->qfout_dev, kQnCap, c->st));
  TRY_HIP(launch_qn_commit(c->qst, c->qxq, c->Wp, c->ppad, c->rp, c->npad, c->p, c->r, c->n,
                           c->Wuser, c->Huser, c->bf16 ? nullptr : c->WT,
                           c->bf16 ? c->WbT : nullptr, c->lwt, c->bf16 ? c->Hb : nullptr, c->st));
  if (c->fuse) {
    TRY_HIP(launch_update_w(c->rp, c->p, c->r, nullptr, 0, 0, 0, nullptr, c->Wp, c->Wuser,
                            nullptr, nullptr, 0, c->bf16, c->gpw, c->uw_grid, c->uw_kpt, true,
                            c->st));
    TRY_HIP(update_h_call(c, nullptr, 0, 0, 0, nullptr, nullptr, c->gph, true));
  } else {
    TRY(gram_h(c));
    TRY(gram_w(c));
  }
  return NMF_OK;
}

// Workspace and graph of QN(q) for this context; the history (rings, their
// Grams, counters) is cleared on every call.
nmf_status qn_prepare(nmf_ctx* c, int q) {
  const int64_t D = qn_dim(c);
  const int qm = qn_max_q();
  if (c->qn_q != q || !c->qn_ws) {
    if (c->qn_graph) (void)hipGraphExecDestroy(c->qn_graph);
    c->qn_graph = nullptr;
    if (c->qn_ws) (void)hipFree(c->qn_ws);
    c->qn_ws = nullptr;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) / 256 * 256;
      return o;
    };
    const size_t ox0 = take(4 * (size_t)D), ox1 = take(4 * (size_t)D), oxq = take(4 * (size_t)D);
    const size_t oU = take(8 * (size_t)q * D), oV = take(8 * (size_t)q * D);
    const size_t odp = take(8 * (size_t)qn_dot_blocks() * 3 * q);
    const size_t oguu = take(8 * (size_t)qm * qm), oguv = take(8 * (size_t)qm * qm);
    const size_t oc = take(8 * (size_t)qm), of = take(8 * 2), ost = take(4 * 8);
    if (hipMalloc(&c->qn_ws, off) != hipSuccess) {
      c->qn_ws = nullptr;
      (void)hipGetLastError();
      return NMF_ENOMEM;
    }
    char* b = static_cast<char*>(c->qn_ws);
    c->qx0 = reinterpret_cast<float*>(b + ox0);
    c->qx1 = reinterpret_cast<float*>(b + ox1);
    c->qxq = reinterpret_cast<float*>(b + oxq);
    c->qU = reinterpret_cast<double*>(b + oU);
    c->qV = reinterpret_cast<double*>(b + oV);
    c->qdpart = reinterpret_cast<double*>(b + odp);
    c->qGUU = reinterpret_cast<double*>(b + oguu);
    c->qGUV = reinterpret_cast<double*>(b + oguv);
    c->qcoef = reinterpret_cast<double*>(b + oc);
    c->qf = reinterpret_cast<double*>(b + of);
    c->qst = reinterpret_cast<int32_t*>(b + ost);
    c->qn_q = q;
    if (!c->qfout) {
      if (hipHostMalloc(reinterpret_cast<void**>(&c->qfout), sizeof(double) * kQnCap,
                        hipHostMallocCoherent) != hipSuccess) {
        c->qfout = nullptr;
        (void)hipGetLastError();
        return NMF_ENOMEM;
      }
      TRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->qfout_dev), c->qfout, 0));
    }
    // one QN iteration as a graph (arguments fixed; per-iteration indices
    // live in device memory)
    if (!c->cap_stream) TRY_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->st;
    const bool prof = c->prof;
    c->prof = false;
    c->st = c->cap_stream;
    hipGraph_t graph = nullptr;
    nmf_status s = NMF_OK;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      s = NMF_EDEVICE;
    if (s == NMF_OK) {
      s = qn_enqueue(c);
      const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
      if (s == NMF_OK && (e != hipSuccess || !graph)) s = NMF_EDEVICE;
    }
    c->st = user;
    c->prof = prof;
    if (s == NMF_OK &&
        (hipGraphInstantiate(&c->qn_graph, graph, nullptr, nullptr, 0) != hipSuccess ||
         hipGraphUpload(c->qn_graph, c->st) != hipSuccess))
      s = NMF_EDEVICE;
    if (graph) (void)hipGraphDestroy(graph);
    if (s != NMF_OK) return s;
  }
  // clear the history: rings, Grams, coefficients, counters (fill kernels)
  const size_t words = ((size_t)(reinterpret_cast<char*>(c->qst) - reinterpret_cast<char*>(c->qU)) +
                        4 * 8) / 4;
  TRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(c->qU), (int64_t)words, 0u, c->st));
  return NMF_OK;
}

nmf_status setup(nmf_ctx* c) {
  const int64_t p = c->p, n = c->n;
  const int rp = c->rp;
  c->ppad = round_up(p, 256);
  c->npad = round_up(n, 256);
  const int64_t ppad = c->ppad, npad = c->npad;
  c->bf16 = (c->opt.precision == NMF_BF16);

  // V as read by the float32 kernels.  The copy ring reads whole tiles, so
  // the FP32 tier uses the caller's buffer only when its rows are 16-byte
  // aligned and p, n are multiples of 256; otherwise (and for misaligned
  // rows in the BF16 tier, whose products read the bf16 shadows) a
  // zero-padded ppad x npad copy.
  const bool aligned = (reinterpret_cast<uintptr_t>(c->Vuser) % 16 == 0) && (c->ldv % 4 == 0);
  const bool bad_pitch = (c->ldv * 4) % 4096 == 0;
  const bool need_copy =
      !aligned || (!c->bf16 && (p % 256 != 0 || n % 256 != 0 || bad_pitch));
  // pad of a pitch that is a multiple of 4 KB, per copy (bytes, multiples of
  // 128, measured per copy at 1024 x 4096 to 8192 x 32768; NMF_PAD_V / _VB /
  // _VT override them)
  const int64_t pad_v = env_int("NMF_PAD_V", 256) / 128 * 128;
  const int64_t pad_vb = env_int("NMF_PAD_VB", 384) / 128 * 128;
  const int64_t pad_vt = env_int("NMF_PAD_VT", 512) / 128 * 128;
  c->ldvk = need_copy ? spread_pitch(npad, 4, pad_v) : c->ldv;
  const int es = c->bf16 ? 2 : 4;
  c->lvb = spread_pitch(npad, 2, pad_vb);
  c->lvt = spread_pitch(ppad, es, pad_vt);
  c->lwt = spread_pitch(ppad, es, pad_vt);

  // tiles and splits (environment overrides are tuning knobs)
  // workgroups the split-K plan aims at: 512 (two per CU) in FP32, 256 in
  // BF16, whose passes stream half the bytes and gain more from half the
  // partials than from the second workgroup per CU (8192 x 32768, rank 256:
  // 158 -> 153 us per pass; 4096 x 16384, ranks 32 and 64: 64.0 -> 61.6 and
  // 90.3 -> 85.6 us per iteration; 8192 x 32768 ranks 32 and 64 unchanged)
  const int64_t target = env_int("NMF_SPLIT_TARGET", c->bf16 ? 256 : 512);
  const int64_t target2 = env_int("NMF_SPLIT_TARGET2", target);
  const int64_t gtarget = env_int("NMF_GRAM_TARGET", 256);
  const int64_t gmin = env_int("NMF_GRAM_MINSTEPS", 8);
  // default tiles, or the narrow ones where the default leaves fewer than
  // 256 workgroups (fewer MFMA waves than SIMDs)
  auto blocks = [](const Split& sp, const DmaCfg& d, int64_t M, int64_t N) {
    return (int64_t)sp.splits * ((M + d.bm - 1) / d.bm) * ((N + d.bn - 1) / d.bn);
  };
  // A tile must divide the padded row counts of both operands it copies
  // (the ring reads whole tiles): pass 1 reads ppad rows of V and rp rows of
  // H, pass 2 rp rows of W^T and npad rows of V^T.  An override that does
  // not fit is ignored.
  auto fits1 = [&](const DmaCfg& d) { return ppad % d.bm == 0 && rp % d.bn == 0; };
  auto fits2 = [&](const DmaCfg& d) { return rp % d.bm == 0 && npad % d.bn == 0; };
  c->d1 = dma_config(rp, true, false, c->bf16);
  c->d2 = dma_config(rp, false, false, c->bf16);
  c->s1 = plan_split(p, rp, npad, c->d1.bm, c->d1.bn, 256, target, 1);
  c->s2 = plan_split(rp, n, ppad, c->d2.bm, c->d2.bn, 256, target2, 1);
  if (blocks(c->s1, c->d1, p, rp) < 256) c->d1 = dma_config(rp, true, true, c->bf16);
  if (blocks(c->s2, c->d2, rp, n) < 256) c->d2 = dma_config(rp, false, true, c->bf16);
  const int64_t id1 = env_int("NMF_DMA1", -1), id2 = env_int("NMF_DMA2", -1);
  if (id1 >= 0 && fits1(dma_config_by_id((int)id1))) c->d1 = dma_config_by_id((int)id1);
  if (id2 >= 0 && fits2(dma_config_by_id((int)id2))) c->d2 = dma_config_by_id((int)id2);
  if (!fits1(c->d1) || !fits2(c->d2)) return NMF_EUNSUPPORTED;
  c->s1 = plan_split(p, rp, npad, c->d1.bm, c->d1.bn, 256, target, 1);
  c->s2 = plan_split(rp, n, ppad, c->d2.bm, c->d2.bn, 256, target2, 1);
  c->kl = (c->opt.loss == NMF_LOSS_POISSON);
  if (c->kl) {
    // every tile holds all padded ranks (pass 1: 128 data rows, pass 2: 128
    // data columns); split-K partials as for the Euclidean passes
    int bm1, bn1, bm2, bn2;
    kl_tiles(rp, &bm1, &bn1, &bm2, &bn2);
    c->s1 = plan_split(p, rp, npad, bm1, bn1, 256, target, 1);
    c->s2 = plan_split(rp, n, ppad, bm2, bn2, 256, target2, 1);
  }
  c->fuse = rp <= 64 && !c->kl;
  // coalesced chunks of 32 elements for the rank-64 Gram (4096 elements:
  // 128 chunks); the smaller Grams have too few chunks to spread over the
  // workgroups and keep one element per 32 lanes (NMF_GRAM_WIDE overrides)
  c->gram_wide = (int)env_int("NMF_GRAM_WIDE", rp >= 64 ? 1 : 0) != 0;
  // where the products reduce the previous update's Gram partials: the
  // coalesced form before their ring loop, under the first copies
  // (4096 x 16384, rank 64: 177.5 -> 175.4 us per iteration; BF16 2048 x
  // 8192: 40.0 -> 38.7 us), the per-element form after it (rank 16: 17.4
  // against 17.6 us; before the coalesced form, at rank 64 too: 83.7 ->
  // 80.7 us per pass); NMF_GRAM_AT_END overrides
  c->gram_at_end = (int)env_int("NMF_GRAM_AT_END", c->gram_wide ? 0 : 1) != 0;
  if (!c->fuse && !c->kl) {
    if (!c->bf16) {
      c->cgh = nt_config(rp, true);
      c->cgw = tn_config(rp, true);
      c->sgh = plan_split(rp, rp, n, c->cgh.bm, c->cgh.bn, c->cgh.bk, gtarget, gmin);
      c->sgw = plan_split(rp, rp, p, c->cgw.bm, c->cgw.bn, c->cgw.bk, gtarget, gmin);
    } else {
      c->cgh = nt_bf16_config(rp, true);
      c->sgh = plan_split(rp, rp, n, c->cgh.bm, c->cgh.bn, c->cgh.bk_bf16, gtarget, gmin);
      c->sgw = plan_split(rp, rp, p, c->cgh.bm, c->cgh.bn, c->cgh.bk_bf16, gtarget, gmin);
    }
  }
  c->nparts = objective_parts(p, n);
  const int ucap = c->fuse ? (int)env_int("NMF_UPDATE_CAP", 512) : 0;
  c->uw_kpt = update_w_kpt(rp, p);
  c->uh_cols = update_h_cols(n);
  const int64_t kpt_env = env_int("NMF_UW_KPT", 0), cols_env = env_int("NMF_UH_COLS", 0);
  if (kpt_env == 1 || kpt_env == 4) c->uw_kpt = (int)kpt_env;
  if (cols_env == 16 || cols_env == 32 || cols_env == 64) c->uh_cols = (int)cols_env;
  c->uw_grid = update_grid(rp, p, ucap, c->uw_kpt);
  c->uh_grid = update_h_grid(n, ucap, c->uh_cols);

  // carve one allocation, 256-byte aligned pieces
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t oVc = need_copy ? take(sizeof(float) * (size_t)ppad * c->ldvk) : 0;
  const size_t oWp = take(sizeof(float) * (size_t)ppad * rp);
  const size_t oHp = take(sizeof(float) * (size_t)rp * npad);
  const size_t oGH = take(sizeof(float) * (size_t)rp * rp);
  const size_t oGW = take(sizeof(float) * (size_t)rp * rp);
  const size_t o1 = take(sizeof(float) * (size_t)c->s1.splits * c->s1.sp);
  const size_t o2 = take(sizeof(float) * (size_t)c->s2.splits * c->s2.sp);
  const size_t og = (c->fuse || c->kl) ? 0
                            : take(sizeof(float) * std::max((size_t)c->sgh.splits * c->sgh.sp,
                                                            (size_t)c->sgw.splits * c->sgw.sp));
  const size_t ogw = c->fuse ? take(sizeof(float) * (size_t)c->uw_grid * rp * rp) : 0;
  const size_t ogh = c->fuse ? take(sizeof(float) * (size_t)c->uh_grid * rp * rp) : 0;
  const size_t ofp = take(sizeof(double) * (size_t)c->nparts);
  const size_t ofl = take(sizeof(uint32_t) * 4);
  const size_t oli = c->fuse ? take(sizeof(double) * (size_t)rp * rp) : 0;
  const size_t okl = c->kl ? take(sizeof(float) * 2 * (size_t)rp) : 0;
  size_t oVT = 0, oWT = 0, oVb = 0, oVTb = 0, oHb = 0, oWbT = 0;
  if (!c->bf16) {
    oVT = take(sizeof(float) * (size_t)npad * c->lvt);
    oWT = take(sizeof(float) * (size_t)rp * c->lwt);
  } else {
    oVb = take(sizeof(uint16_t) * (size_t)ppad * c->lvb);
    oVTb = take(sizeof(uint16_t) * (size_t)npad * c->lvt);
    oHb = take(sizeof(uint16_t) * (size_t)rp * npad);
    oWbT = take(sizeof(uint16_t) * (size_t)rp * c->lwt);
  }
  if (hipMalloc(&c->ws, off) != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return NMF_ENOMEM;
  }
  char* base = static_cast<char*>(c->ws);
  if (need_copy) c->Vcopy = reinterpret_cast<float*>(base + oVc);
  c->Wp = reinterpret_cast<float*>(base + oWp);
  c->Hp = reinterpret_cast<float*>(base + oHp);
  c->GH = reinterpret_cast<float*>(base + oGH);
  c->GW = reinterpret_cast<float*>(base + oGW);
  c->part1 = reinterpret_cast<float*>(base + o1);
  c->part2 = reinterpret_cast<float*>(base + o2);
  if (!c->fuse && !c->kl) c->partg = reinterpret_cast<float*>(base + og);
  if (c->fuse) {
    c->gpw = reinterpret_cast<float*>(base + ogw);
    c->gph = reinterpret_cast<float*>(base + ogh);
  }
  c->fpart = reinterpret_cast<double*>(base + ofp);
  c->flag = reinterpret_cast<uint32_t*>(base + ofl);
  if (c->fuse) c->lsinv = reinterpret_cast<double*>(base + oli);
  if (c->kl) c->kl_den = reinterpret_cast<float*>(base + okl);
  if (!c->bf16) {
    c->VT = reinterpret_cast<float*>(base + oVT);
    c->WT = reinterpret_cast<float*>(base + oWT);
  } else {
    c->Vb = reinterpret_cast<uint16_t*>(base + oVb);
    c->VTb = reinterpret_cast<uint16_t*>(base + oVTb);
    c->Hb = reinterpret_cast<uint16_t*>(base + oHb);
    c->WbT = reinterpret_cast<uint16_t*>(base + oWbT);
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->hostbuf), 4 * sizeof(double),
                    hipHostMallocCoherent) != hipSuccess) {
    c->hostbuf = nullptr;
    (void)hipGetLastError();
    return NMF_ENOMEM;
  }
  TRY_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->hostbuf_dev), c->hostbuf, 0));
  for (hipEvent_t& e : c->chk_ev) TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));

  // zero the whole workspace (padding must read as zero)
  TRY_HIP(launch_fill_u32(static_cast<uint32_t*>(c->ws), (int64_t)(off / 4), 0u, c->st));

  if (c->opt.validate) {
    TRY_HIP(launch_validate(c->Vuser, c->ldv, p, n, c->flag, c->st));
    TRY_HIP(hipMemcpyAsync(c->hostbuf, c->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->st));
    TRY_HIP(hipStreamSynchronize(c->st));
    uint32_t bad;
    std::memcpy(&bad, c->hostbuf, sizeof(bad));
    if (bad) return NMF_EINVAL;
  }

  if (need_copy) {
    TRY_HIP(launch_copy_pad(c->Vuser, c->ldv, p, n, c->Vcopy, c->ldvk, c->st));
    c->Vk = c->Vcopy;
  } else {
    c->Vk = c->Vuser;
  }

  if (c->opt.seed != 0) {
    TRY_HIP(launch_uniform(c->Wuser, p, c->r, c->r, c->opt.seed, 0u, c->st));
    TRY_HIP(launch_uniform(c->Huser, c->r, n, n, c->opt.seed, 1u, c->st));
  }
  TRY_HIP(launch_copy_pad(c->Wuser, c->r, p, c->r, c->Wp, rp, c->st));
  TRY_HIP(launch_copy_pad(c->Huser, n, c->r, n, c->Hp, npad, c->st));

  if (!c->bf16) {
    TRY_HIP(launch_transpose_f32(c->Vk, c->ldvk, p, n, c->VT, c->lvt, c->st));
    TRY_HIP(launch_transpose_f32(c->Wp, rp, ppad, rp, c->WT, c->lwt, c->st));
  } else {
    TRY_HIP(launch_cast_bf16(c->Vk, c->ldvk, p, n, c->Vb, c->lvb, false, c->st));
    TRY_HIP(launch_cast_bf16(c->Vk, c->ldvk, p, n, c->VTb, c->lvt, true, c->st));
    TRY_HIP(launch_cast_bf16(c->Hp, npad, rp, npad, c->Hb, npad, false, c->st));
    TRY_HIP(launch_cast_bf16(c->Wp, rp, ppad, rp, c->WbT, c->lwt, true, c->st));
  }

  // ||V||_F^2 (objective with W = 0), then the Grams of the start
  TRY(objective_sync(c, nullptr, &c->nv2));
  if (c->fuse) {
    // per-workgroup Grams of the start; the first products reduce them
    TRY_HIP(launch_update_w(rp, p, c->r, nullptr, 0, 0, 0, nullptr, c->Wp, c->Wuser, nullptr,
                            nullptr, 0, c->bf16, c->gpw, c->uw_grid, c->uw_kpt, true, c->st));
    TRY_HIP(update_h_call(c, nullptr, 0, 0, 0, nullptr, nullptr, c->gph, true));
  } else if (!c->kl) {
    TRY(gram_h(c));
    TRY(gram_w(c));
  }
  return NMF_OK;
}

}  // namespace

extern "C" {

void nmf_default_options(nmf_options* opt) {
  if (!opt) return;
  opt->precision = NMF_FP32;
  opt->tol_kind = NMF_TOL_REL_CHANGE;
  opt->tol = 1e-9;
  opt->check_every = 1;
  opt->validate = 0;
  opt->seed = 0;
  opt->use_graph = 1;
  opt->loss = NMF_LOSS_EUCLIDEAN;
}

nmf_status nmf_init(nmf_ctx** out, const float* V, int64_t p, int64_t n, int64_t ldv, int32_t r,
                    float* W, float* H, const nmf_options* opt, void* stream) {
  if (!out) return NMF_EINVAL;
  *out = nullptr;
  nmf_options o;
  nmf_default_options(&o);
  if (opt) o = *opt;
  if (p <= 0 || n <= 0 || r <= 0 || ldv < n) return NMF_EINVAL;
  TRY(check_ptr(V));
  TRY(check_ptr(W));
  TRY(check_ptr(H));
  if (o.check_every < 1 || !(o.tol >= 0.0) || !std::isfinite(o.tol)) return NMF_EINVAL;
  if (o.precision != NMF_FP32 && o.precision != NMF_BF16) return NMF_EUNSUPPORTED;
  if (o.tol_kind != NMF_TOL_REL_CHANGE && o.tol_kind != NMF_TOL_GAP_NORMALIZED)
    return NMF_EUNSUPPORTED;
  if (o.loss != NMF_LOSS_EUCLIDEAN && o.loss != NMF_LOSS_POISSON) return NMF_EUNSUPPORTED;
  if (r > NMF_MAX_RANK || p > kMaxDim || n > kMaxDim) return NMF_EUNSUPPORTED;
  // the Poisson update: float32, padded rank <= 64, relative-change rule
  if (o.loss == NMF_LOSS_POISSON &&
      (o.precision != NMF_FP32 || r > 64 || o.tol_kind != NMF_TOL_REL_CHANGE))
    return NMF_EUNSUPPORTED;

  nmf_ctx* c = new (std::nothrow) nmf_ctx();
  if (!c) return NMF_ENOMEM;
  c->st = static_cast<hipStream_t>(stream);
  c->p = p;
  c->n = n;
  c->ldv = ldv;
  c->r = r;
  c->rp = padded_rank(r);
  c->opt = o;
  c->Vuser = V;
  c->Wuser = W;
  c->Huser = H;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
          hipSuccess) {
    (void)hipGetLastError();
    free_ctx(c);
    return NMF_EDEVICE;
  }
  nmf_status s = setup(c);
  if (s != NMF_OK) {
    (void)hipStreamSynchronize(c->st);
    free_ctx(c);
    return s;
  }
  *out = c;
  return NMF_OK;
}

nmf_status nmf_update_w(nmf_ctx* c) {
  if (!c) return NMF_EINVAL;
  if (c->kl) return NMF_EUNSUPPORTED;  // the Poisson update has no half-steps
  return half_w(c);
}

nmf_status nmf_update_h(nmf_ctx* c) {
  if (!c) return NMF_EINVAL;
  if (c->kl) return NMF_EUNSUPPORTED;
  return half_h(c);
}

nmf_status nmf_step(nmf_ctx* c, int32_t iters) {
  if (!c || iters < 0) return NMF_EINVAL;
  if (!c->opt.use_graph || c->prof) {
    for (int32_t it = 0; it < iters; ++it) TRY(iterate(c));
    return NMF_OK;
  }
  // the largest graph while it fits, then the binary digits of the rest
  // (10 iterations = one launch of 8 and one of 2)
  constexpr int top = kGraphLevels - 1;
  int32_t left = iters;
  for (int j = top; j >= 0; --j) {
    const int32_t n = 1 << j;
    while (left >= n) {
      if (!c->gp[j]) TRY(capture(c, n, &c->gp[j]));
      TRY_HIP(hipGraphLaunch(c->gp[j], c->st));
      left -= n;
      if (j < top) break;
    }
  }
  return NMF_OK;
}

nmf_status nmf_prepare_graphs(nmf_ctx* c) {
  if (!c) return NMF_EINVAL;
  if (!c->opt.use_graph) return NMF_OK;
  for (int j = 0; j < kGraphLevels; ++j)
    if (!c->gp[j]) TRY(capture(c, 1 << j, &c->gp[j]));
  return NMF_OK;
}

nmf_status nmf_objective(nmf_ctx* c, double* f_host) {
  if (!c || !f_host) return NMF_EINVAL;
  double f;
  TRY(objective_sync(c, c->Wp, &f));
  *f_host = f;
  return std::isfinite(f) ? NMF_OK : NMF_ENONFINITE;
}

namespace {

// Objective of the state after everything enqueued so far, written into
// check slot `slot` (hostbuf[2 + slot]); chk_ev[slot] marks its arrival.
nmf_status enqueue_check(nmf_ctx* c, int slot) {
  TRY(objective_async(c, c->Wp, c->hostbuf_dev + 2 + slot));
  TRY_HIP(hipEventRecord(c->chk_ev[slot], c->st));
  return NMF_OK;
}

nmf_status wait_check(nmf_ctx* c, int slot, double* f) {
  TRY_HIP(hipEventSynchronize(c->chk_ev[slot]));
  *f = c->hostbuf[2 + slot];
  return NMF_OK;
}

}  // namespace

nmf_status nmf_solve(nmf_ctx* c, int32_t max_iters, int32_t* iters_done, double* f_host,
                     double* trace, int32_t trace_len) {
  if (!c || max_iters < 0 || !iters_done || !f_host) return NMF_EINVAL;
  if (trace && trace_len < 0) return NMF_EINVAL;
  double f_prev;
  *iters_done = 0;
  nmf_status s = nmf_objective(c, &f_prev);
  *f_host = f_prev;
  if (s != NMF_OK) return s;
  int32_t nt = 0;
  if (trace && nt < trace_len) trace[nt++] = f_prev;
  if (max_iters == 0) return NMF_ENOTCONVERGED;

  // Chunks of check_every iterations, each followed by an objective whose
  // value is copied to the host.  The next chunk and its check are enqueued
  // before the host waits for the current check, so the device never idles
  // on the host; the price is that when the rule holds, the chunk already
  // enqueued after that check also runs (and its objective is the final
  // one: the value returned always belongs to the factors returned).
  int32_t queued = 0;         // iterations enqueued
  int32_t pend_k[2] = {0, 0};  // iterations behind each pending check
  int head = 0, npend = 0;    // oldest pending slot, pending count
  auto push = [&]() -> nmf_status {
    const int32_t todo = std::min(c->opt.check_every, max_iters - queued);
    TRY(nmf_step(c, todo));
    queued += todo;
    const int slot = (head + npend) & 1;
    TRY(enqueue_check(c, slot));
    pend_k[slot] = queued;
    ++npend;
    return NMF_OK;
  };
  TRY(push());
  bool done = false;
  while (npend > 0) {
    if (!done && queued < max_iters && npend < 2) TRY(push());
    double f;
    TRY(wait_check(c, head, &f));
    *iters_done = pend_k[head];
    *f_host = f;
    head ^= 1;
    --npend;
    if (trace && nt < trace_len) trace[nt++] = f;
    if (!std::isfinite(f)) {
      s = NMF_ENONFINITE;
      done = true;
      continue;  // drain the pending check (its factors are the returned ones)
    }
    if (done) continue;
    if (c->opt.tol_kind == NMF_TOL_REL_CHANGE)
      done = std::fabs(f - f_prev) / (std::fabs(f_prev) + 1.0) < c->opt.tol;
    else
      done = (c->nv2 > 0.0 ? f / c->nv2 : 0.0) <= c->opt.tol;
    f_prev = f;
  }
  if (s == NMF_ENONFINITE) return s;
  return done ? NMF_OK : NMF_ENOTCONVERGED;
}

nmf_status nmf_solve_qn(nmf_ctx* c, int32_t q, int32_t max_iters, int32_t* iters_done,
                        int32_t* accepted, double* f_host, double* trace, int32_t trace_len) {
  if (!c || !iters_done || !f_host || q < 1 || max_iters < 0) return NMF_EINVAL;
  if (trace && trace_len < 0) return NMF_EINVAL;
  if (q > qn_max_q() || max_iters / 2 > kQnCap) return NMF_EINVAL;
  if (c->kl) return NMF_EUNSUPPORTED;
  if (c->Hp != c->Wp + c->ppad * c->rp) return NMF_EUNSUPPORTED;  // [Wp | Hp] contiguous
  *iters_done = 0;
  if (accepted) *accepted = 0;
  double f_prev;
  nmf_status s = nmf_objective(c, &f_prev);
  *f_host = f_prev;
  if (s != NMF_OK) return s;
  int32_t nt = 0;
  if (trace && nt < trace_len) trace[nt++] = f_prev;
  TRY(qn_prepare(c, q));
  // chunks of check_every map evaluations (check_every / 2 QN iterations,
  // at least one); the rule is tested on the accepted objective at the end
  // of each chunk
  const int32_t chunk = std::max<int32_t>(1, c->opt.check_every / 2);
  const int32_t total = max_iters / 2;
  int32_t it = 0;
  bool done = false;
  double f = f_prev;
  while (!done && it < total) {
    const int32_t todo = std::min(chunk, total - it);
    for (int32_t k = 0; k < todo; ++k) TRY_HIP(hipGraphLaunch(c->qn_graph, c->st));
    TRY_HIP(hipStreamSynchronize(c->st));
    for (int32_t k = it; k < it + todo; ++k)
      if (trace && nt < trace_len) trace[nt++] = c->qfout[k];
    it += todo;
    f = c->qfout[it - 1];
    if (!std::isfinite(f)) {
      s = NMF_ENONFINITE;
      break;
    }
    if (c->opt.tol_kind == NMF_TOL_REL_CHANGE)
      done = std::fabs(f - f_prev) / (std::fabs(f_prev) + 1.0) < c->opt.tol;
    else
      done = (c->nv2 > 0.0 ? f / c->nv2 : 0.0) <= c->opt.tol;
    f_prev = f;
  }
  *iters_done = 2 * it;
  *f_host = f;
  if (accepted) {
    int32_t* st = reinterpret_cast<int32_t*>(c->hostbuf);  // pinned
    TRY_HIP(hipMemcpyAsync(st, c->qst, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    TRY_HIP(hipStreamSynchronize(c->st));
    *accepted = st[1];
  }
  if (s != NMF_OK) return s;
  return done ? NMF_OK : NMF_ENOTCONVERGED;
}

nmf_status nmf_refit_w(nmf_ctx* c, float floor_rel) {
  if (!c || !(floor_rel > 0.f && floor_rel < 1.f)) return NMF_EINVAL;
  if (c->kl || !c->fuse || c->rp > 64) return NMF_EUNSUPPORTED;
  // A = V H^T as in the W half-step; the same launch reduces G_H
  const GramRed gr = GramRed{c->gph, c->uh_grid, c->rp * c->rp, c->GH, 0, c->gram_wide};
  const void* X = c->bf16 ? static_cast<const void*>(c->Vb) : static_cast<const void*>(c->Vk);
  const void* Y = c->bf16 ? static_cast<const void*>(c->Hb) : static_cast<const void*>(c->Hp);
  TRY_HIP(launch_nt_dma(c->d1, c->bf16, X, c->bf16 ? c->lvb : c->ldvk, c->p, Y, c->npad, c->rp,
                        c->npad, c->s1.splits, c->s1.kchunk, c->part1, c->s1.ldp, c->s1.sp, gr,
                        c->st));
  TRY_HIP(launch_ls_refit(c->GH, c->rp, c->r, c->p, c->part1, c->s1.ldp, c->s1.sp, c->s1.splits,
                          c->lsinv, c->flag + 1, floor_rel, c->Wp, c->Wuser, c->st));
  return NMF_OK;
}

nmf_status nmf_data_norm2(nmf_ctx* c, double* norm2_host) {
  if (!c || !norm2_host) return NMF_EINVAL;
  *norm2_host = c->nv2;
  return NMF_OK;
}

nmf_status nmf_profile_start(nmf_ctx* c, int32_t max_records) {
  if (!c || max_records < 1) return NMF_EINVAL;
  TRY_HIP(hipStreamSynchronize(c->st));
  profile_release(c);
  c->ev.assign(2 * (size_t)max_records, nullptr);
  c->ev_stage.assign((size_t)max_records, 0);
  for (size_t i = 0; i < c->ev.size(); ++i) {
    if (hipEventCreate(&c->ev[i]) != hipSuccess) {
      c->ev.resize(i);
      profile_release(c);
      return NMF_EDEVICE;
    }
  }
  c->prof_cap = max_records;
  c->prof_used = 0;
  c->prof = true;
  return NMF_OK;
}

nmf_status nmf_profile_stop(nmf_ctx* c, double* ms_host, int32_t* launches_host) {
  if (!c) return NMF_EINVAL;
  double ms[NMF_STAGE_COUNT] = {0};
  int32_t cnt[NMF_STAGE_COUNT] = {0};
  nmf_status st = NMF_OK;
  if (hipStreamSynchronize(c->st) != hipSuccess) st = NMF_EDEVICE;
  for (int32_t i = 0; st == NMF_OK && i < c->prof_used; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) {
      st = NMF_EDEVICE;
      break;
    }
    ms[c->ev_stage[i]] += t;
    cnt[c->ev_stage[i]] += 1;
  }
  profile_release(c);
  for (int k = 0; k < NMF_STAGE_COUNT; ++k) {
    if (ms_host) ms_host[k] = ms[k];
    if (launches_host) launches_host[k] = cnt[k];
  }
  return st;
}

void nmf_destroy(nmf_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  free_ctx(c);
}

const char* nmf_strerror(nmf_status s) {
  switch (s) {
    case NMF_OK: return "success";
    case NMF_ENOTCONVERGED: return "iteration cap reached before the stopping rule held";
    case NMF_EINVAL: return "invalid argument or invalid data";
    case NMF_ENOMEM: return "device allocation failed";
    case NMF_EDEVICE: return "HIP runtime error";
    case NMF_ENONFINITE: return "objective is not finite";
    case NMF_EUNSUPPORTED: return "unsupported rank, size or option";
  }
  return "unknown status";
}

nmf_status nmf_normalize_gauge(float* W, int64_t p, int32_t r, float* H, int64_t n,
                               void* stream) {
  if (!W || !H || p < 1 || n < 1 || r < 1 || r > NMF_MAX_RANK) return NMF_EINVAL;
  if (reinterpret_cast<uintptr_t>(W) % 4 != 0 || reinterpret_cast<uintptr_t>(H) % 4 != 0)
    return NMF_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* norms = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&norms), sizeof(float) * r, st) != hipSuccess) {
    (void)hipGetLastError();
    return NMF_ENOMEM;
  }
  const hipError_t e = launch_gauge(W, p, r, H, n, norms, st);
  (void)hipFreeAsync(norms, st);
  return e == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

int32_t nmf_version(void) { return 100; }

}  // extern "C"

namespace {

// Scratch of nmf_normalize_gauge_noalloc: the r column norms of W.  Every
// GPU the library runs on holds its own copy at its own address until the
// process ends.  In host code `scratch` names a host-side stand-in, never
// the device memory: kernels get the per-device address that
// hipGetSymbolAddress returns (scratch_on_device below).
__device__ __align__(256) float scratch[NMF_MAX_RANK];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept; nullptr on failure.
float* scratch_on_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

nmf_status nmf_normalize_gauge_noalloc(float* W, int64_t p, int32_t r, float* H, int64_t n,
                                       void* stream) {
  if (!W || !H || p < 1 || n < 1 || r < 1) return NMF_EINVAL;
  if (r > NMF_MAX_RANK) return NMF_EINVAL;  // the scratch holds NMF_MAX_RANK norms
  if (reinterpret_cast<uintptr_t>(W) % 4 != 0 || reinterpret_cast<uintptr_t>(H) % 4 != 0)
    return NMF_EINVAL;
  float* norms = scratch_on_device();
  if (!norms) return NMF_EDEVICE;
  // k_col_norms writes norms[0..r) before k_apply_gauge reads them (same
  // stream), so nothing left by an earlier call is read.
  const hipError_t e = launch_gauge(W, p, r, H, n, norms, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NMF_OK : NMF_EDEVICE;
}

}  // extern "C"
