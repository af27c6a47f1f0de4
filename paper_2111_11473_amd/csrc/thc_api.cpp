// C ABI and host orchestration of the THC-CCSD hot path on one MI355X.
//
// The residual is evaluated as the paper's Algorithms 1-3 and 8 fused into one pass over
// blocks of Cholesky vectors, Algorithm 6 (quartic T2^2 terms, H-kernel), Algorithm 7 (T2^2
// rings), Algorithms 9-10 and the projection onto the working basis.  Every contraction is
// a launch of the library's FP64 MFMA GEMM or of one of its elementwise kernels; the host
// only sequences launches on one stream and reads back scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/thc.h"
#include "internal.h"

using namespace thc;

namespace {

constexpr int64_t GEMM_WS = int64_t(1) << 22;  // 32 MB
// generator streams of the synthetic inputs (the order of the Python generator)
constexpr uint64_t thc_synth_stream_xo_amp = 3, thc_synth_stream_xv_amp = 4, thc_synth_stream_xo_eri = 5,
                   thc_synth_stream_xv_eri = 6;

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
  int64_t launches;  // kernel dispatches between a and b
};

struct Buf {
  double* p = nullptr;
  size_t n = 0;
};

}  // namespace

struct thc_ctx {
  thc_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  bool built = false;

  int64_t o = 0, v = 0, n = 0, nL = 0, P = 0, Q = 0, Pp = 0, ov = 0;
  // synthetic inputs generated on the device (thc_set_synthetic)
  bool synth = false;
  thc_synth_spec spec{};
  double gamma = 0.0;         // global scale of the Cholesky vectors in use
  bool lvv_resident = true;   // the vv Cholesky block is held; else regenerated per fused-pass block
  int64_t nb = 0, KS = 1, Xb = 0, Ic = 0, Xc = 0, X7 = 0;

  std::vector<void*> allocs;
  size_t bytes = 0;
  void* ws = nullptr;            // caller's device workspace (thc_create_with_workspace), or null
  size_t ws_bytes = 0;
  double* arena = nullptr;       // every buffer of the context lies in here
  double* setup_scratch = nullptr;  // scratch of the set-up (overlays the Alg. 6 region)
  size_t setup_len = 0;             // doubles

  // factors (device)
  double *Loo = nullptr, *Lov = nullptr, *Lvv = nullptr, *eps = nullptr;
  double *Yo = nullptr, *Yv = nullptr, *xo = nullptr, *xv = nullptr;
  double *Go = nullptr, *Gv = nullptr, *S = nullptr, *z = nullptr, *Bq = nullptr, *Bkr = nullptr;
  double *W = nullptr, *e = nullptr;
  // state
  double *Th = nullptr, *t1 = nullptr, *Zs = nullptr;
  double* Th0 = nullptr;  // the MP2 guess in the working basis: the solver's fallback start
  // DIIS ring
  double *dvec = nullptr, *derr = nullptr, *dT = nullptr, *dt1 = nullptr;
  int diis_n = 0, diis_head = 0;
  std::vector<double> diisB;  // host copy of the error inner products (diis_max^2)
  double E_last = 0.0;        // energy of the last iteration, for the next call's |dE| test
  bool have_last = false;     // E_last belongs to the current state's iteration history

  // residual outputs
  double *sig = nullptr, *sig1 = nullptr, *sigh = nullptr, *scal = nullptr;

  // A-pass work
  double *Lhoo = nullptr, *Lhvo = nullptr, *tmpoo = nullptr, *tmpooT = nullptr, *Pv = nullptr, *PvT = nullptr;
  double *LovYv = nullptr, *Wv = nullptr, *Bvv = nullptr, *Woo = nullptr, *Boo = nullptr;
  double *Ccat = nullptr, *Dcat = nullptr, *Wvo = nullptr, *Y1 = nullptr, *Gm = nullptr, *GY = nullptr;
  double *TA = nullptr, *tmpov = nullptr;
  double *sig28 = nullptr, *C3 = nullptr, *Abar = nullptr, *At = nullptr, *Hh = nullptr;
  double *xioo = nullptr, *xivv = nullptr, *s38 = nullptr, *dvecA = nullptr, *trK = nullptr;
  double *ej = nullptr, *ek = nullptr;
  double *Fin = nullptr, *Fh = nullptr;  // n x n, blocks [oo | ov | vo | vv]
  double *Jov = nullptr, *Jvo = nullptr;
  // assembly
  double *ST = nullptr, *Dt = nullptr, *K29 = nullptr, *Qm = nullptr, *ot = nullptr, *vt = nullptr, *E9 = nullptr;
  double *tmpoP = nullptr, *tmpvP = nullptr, *Fxoo = nullptr, *Fxvv = nullptr, *Tf = nullptr, *fd = nullptr;
  // Alg. 6
  double *C6 = nullptr, *D6 = nullptr, *Ec = nullptr, *Fc = nullptr, *Gc = nullptr, *GYc = nullptr, *Hb = nullptr;
  // Alg. 4 and 5 (the O(N^5) form of Eq. 32 and 33), when chosen instead of Alg. 6
  bool quintic = false;
  int64_t nq = 0, jq = 0;  // pairs per batched product; occupied j per chunk of the dense residual
  double *Wq = nullptr, *qC = nullptr, *qD1 = nullptr, *qE = nullptr, *qF1 = nullptr, *qF = nullptr, *qG1 = nullptr,
         *qG = nullptr, *qI1 = nullptr, *qR = nullptr, *qT1 = nullptr;
  double* delta = nullptr;     // Jacobi denominator shift of the learned guess (nP)
  void* pin = nullptr;         // pinned host staging buffer for every host <-> device transfer
  size_t pin_bytes = 0;
  bool mixed = false;          // the residual being evaluated uses FP32 MFMA / FP32 H operands
  bool want_mixed = false;     // requested precision of the next residual evaluation
  float *Ec32 = nullptr, *Fc32 = nullptr;  // FP32 H-kernel operands (mixed precision only)
  bool has_shift = false;
  uint32_t* htiles = nullptr;  // H-kernel tile table
  int64_t nhtiles = 0, hslots = 0, hfilled = 0;  // table length (with empty slots), slots per XCD, tiles
  uint32_t* htiles32 = nullptr;  // tile table of the FP32 H-kernel (mixed precision: 16 x 16 block pairs)
  int64_t nhtiles32 = 0, hslots32 = 0;
  float* G32 = nullptr;  // FP32 G (mixed precision), in the FP64 G buffer
  int alg1_tile = 64;          // tile edge of the symmetric Alg. 1 product
  double *R1 = nullptr, *I6 = nullptr;
  // Alg. 7
  double *U7 = nullptr, *S7 = nullptr, *R7 = nullptr, *Rx = nullptr, *Sx = nullptr, *Cx = nullptr, *Dx = nullptr;
  double *F7 = nullptr, *Gt = nullptr, *Gts = nullptr, *G7 = nullptr, *G7s = nullptr;
  double* gws = nullptr;  // split-K workspace of the GEMMs (GEMM_WS doubles)

  // per-iteration history of the last thc_iterate call
  std::vector<double> hist_e, hist_r, hist_t;
  std::vector<int> hist_mixed;  // 1 where the iteration's residual was mixed precision
  std::vector<int> hist_flags;  // THC_ITER_* bits per iteration

  // profiling
  bool prof = false;
  std::vector<ProfRec> recs;
  const char* section = nullptr;  // residual section, for per-section GEMM records ("gemm@<section>")
  int chain = -1;                 // THC_CHAIN_* bit index of the section (split_mask), -1 outside
  thc_mlp* guess_net = nullptr;   // network of the learned start (thc_options.guess = 1), not owned
  bool guess_pending = false;     // the state is the MP2 guess thc_build_factors left
  double gemm_flops = 0.0, gemm_flops32 = 0.0, gemm_flops16 = 0.0;  // MFMA GEMM flops (2 K per distinct output,
                                                                     // FP64 / FP32 / split-BF16) while profiling
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

namespace {

constexpr double C_D = 0.5;  // prefactor of the Eq. 35-37 ring contraction (closed-shell CCSD)

// THC_FLAG_CHECK: every device step is waited for, so an error is reported by the step that
// caused it (the network object has no such mode)
inline hipError_t step_check(thc_ctx* c) {
  return (c->opt.flags & THC_FLAG_CHECK) ? hipStreamSynchronize(c->stream) : hipSuccess;
}
inline hipError_t step_check(thc_mlp*) { return hipSuccess; }

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e == hipSuccess) _e = step_check(ctx);                                      \
    if (_e != hipSuccess) {                                                          \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(_e);                  \
      return THC_EDEVICE;                                                            \
    }                                                                                \
  } while (0)

#define RCHK(expr)                 \
  do {                             \
    int _r = (expr);               \
    if (_r != THC_OK) return _r;   \
  } while (0)

// Host <-> device transfers go through one pinned staging buffer (grown on demand) and complete
// before returning: the caller's host memory is plain pageable memory.
template <class Ctx>
void* pinned(Ctx* ctx, size_t bytes) {
  if (bytes > ctx->pin_bytes) {
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    ctx->pin = nullptr;
    ctx->pin_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&ctx->pin, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ctx->pin = nullptr;
      return nullptr;
    }
    ctx->pin_bytes = want;
  }
  return ctx->pin;
}

template <class Ctx>
int d2h(Ctx* ctx, void* host, const void* dev, size_t bytes) {
  if (bytes == 0) return THC_OK;
  void* p = pinned(ctx, bytes);
  if (!p) { ctx->err = "pinned staging allocation failed"; return THC_ENOMEM; }
  HIPCHK(hipMemcpyAsync(p, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(host, p, bytes);
  return THC_OK;
}

template <class Ctx>
int h2d(Ctx* ctx, void* dev, const void* host, size_t bytes) {
  if (bytes == 0) return THC_OK;
  void* p = pinned(ctx, bytes);
  if (!p) { ctx->err = "pinned staging allocation failed"; return THC_ENOMEM; }
  std::memcpy(p, host, bytes);
  HIPCHK(hipMemcpyAsync(dev, p, bytes, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return THC_OK;
}

// rows x cols block of doubles with device row pitch ld (elements) <-> packed host rows
int d2h_block(thc_ctx* ctx, double* host, const double* dev, int64_t ld, int64_t rows, int64_t cols);
int h2d_block(thc_ctx* ctx, double* dev, int64_t ld, const double* host, int64_t rows, int64_t cols);

hipEvent_t next_event(thc_ctx* ctx) {
  if (ctx->pool_used == ctx->pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    ctx->pool.push_back(ev);
  }
  return ctx->pool[ctx->pool_used++];
}

struct Scope {
  thc_ctx* ctx;
  hipEvent_t a = nullptr;
  const char* name;
  int64_t launches = 1;
  Scope(thc_ctx* c, const char* nm) : ctx(c), name(nm) {
    if (ctx->prof) {
      a = next_event(ctx);
      if (a) (void)hipEventRecord(a, ctx->stream);
    }
  }
  ~Scope() {
    if (ctx->prof && a) {
      hipEvent_t b = next_event(ctx);
      if (b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->recs.push_back({name, a, b, launches});
      }
    }
  }
};

int gemm(thc_ctx* ctx, const Gemm& g0) {
  Scope sc(ctx, "gemm");
  Gemm g = g0;
  g.ws = ctx->gws;
  g.ws_len = ctx->gws ? GEMM_WS : 0;
  if (ctx->mixed && !g.keep64) {
    const bool split = ctx->opt.precision == 2 || (ctx->chain >= 0 && ((ctx->opt.split_mask >> ctx->chain) & 1u));
    if (split) g.bf16x3 = true; else g.f32 = true;
  }
  if (ctx->prof && g.K > 0) {
    // a symmetric product (upper) needs only the N (N + 1) / 2 distinct outputs
    const double outs = g.upper ? 0.5 * g.N * (g.N + 1.0) : (double)g.M * g.N;
    (g.bf16x3 ? ctx->gemm_flops16 : g.f32 ? ctx->gemm_flops32 : ctx->gemm_flops) += 2.0 * outs * g.K * g.batch;
  }
  if (ctx->prof && ctx->section) {
    Scope sc2(ctx, ctx->section);
    HIPCHK(gemm_f64(g, ctx->stream));
  } else {
    HIPCHK(gemm_f64(g, ctx->stream));
  }
  return THC_OK;
}

// Marks a product that stays FP64 in the mixed-precision path (energy partials, T1 dressing).
Gemm k64(Gemm g) {
  g.keep64 = true;
  return g;
}

// Sets the precision for one residual evaluation and restores FP64 on every exit.
struct MixedScope {
  thc_ctx* ctx;
  MixedScope(thc_ctx* c) : ctx(c) { ctx->mixed = ctx->want_mixed; }
  ~MixedScope() {
    ctx->mixed = false;
    ctx->chain = -1;
  }
};

// Plain (batched) GEMM helper.
Gemm mk(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, bool tA, const double* B, int64_t ldb,
        bool tB, double* C, int64_t ldc, double alpha = 1.0, double beta = 0.0) {
  Gemm g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.transA = tA;
  g.B = B; g.ldb = ldb; g.transB = tB;
  g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  return g;
}
Gemm batched(Gemm g, int64_t batch, int64_t sA, int64_t sB, int64_t sC) {
  g.batch = batch; g.sA = sA; g.sB = sB; g.sC = sC;
  return g;
}

#define MISC(expr)                      \
  do {                                  \
    Scope _sc(ctx, "misc");             \
    HIPCHK(expr);                       \
  } while (0)

int zero(thc_ctx* ctx, double* p, size_t count) {
  MISC(k_fill((int64_t)count, 0.0, p, ctx->stream));
  return THC_OK;
}

// ---------------------------------------------------------------------------------------
// Dense SPD solves on the device: blocked right-looking Cholesky (lower, in place) whose
// 64 x 64 diagonal blocks are factored and inverted on the host; the panel and trailing
// updates are GEMMs.  Linv receives the inverses of the diagonal blocks.
constexpr int64_t CB = 64;

int d2h_block(thc_ctx* ctx, double* host, const double* dev, int64_t ld, int64_t rows, int64_t cols) {
  const size_t bytes = (size_t)(rows * cols) * sizeof(double);
  void* p = pinned(ctx, bytes);
  if (!p) { ctx->err = "pinned staging allocation failed"; return THC_ENOMEM; }
  HIPCHK(hipMemcpy2DAsync(p, cols * sizeof(double), dev, ld * sizeof(double), cols * sizeof(double), rows,
                          hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(host, p, bytes);
  return THC_OK;
}

int h2d_block(thc_ctx* ctx, double* dev, int64_t ld, const double* host, int64_t rows, int64_t cols) {
  const size_t bytes = (size_t)(rows * cols) * sizeof(double);
  void* p = pinned(ctx, bytes);
  if (!p) { ctx->err = "pinned staging allocation failed"; return THC_ENOMEM; }
  std::memcpy(p, host, bytes);
  HIPCHK(hipMemcpy2DAsync(dev, ld * sizeof(double), p, cols * sizeof(double), cols * sizeof(double), rows,
                          hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return THC_OK;
}

int potrf(thc_ctx* ctx, double* A, int64_t n, double* Linv, double* tmp, const char* what) {
  std::vector<double> hb(CB * CB), hi(CB * CB);
  for (int64_t k0 = 0; k0 < n; k0 += CB) {
    const int64_t kb = std::min(CB, n - k0);
    RCHK(d2h_block(ctx, hb.data(), A + k0 * n + k0, n, kb, kb));
    if (host_cholesky(kb, hb.data()) != 0) {
      char buf[160];
      snprintf(buf, sizeof buf, "%s is not positive definite (Cholesky pivot <= 0 in diagonal block %lld of %lld)",
               what, (long long)(k0 / CB), (long long)((n + CB - 1) / CB));
      ctx->err = buf;
      return THC_ESINGULAR;
    }
    host_tri_inverse_lower(kb, hb.data(), hi.data());
    RCHK(h2d_block(ctx, A + k0 * n + k0, n, hb.data(), kb, kb));
    double* Li = Linv + (k0 / CB) * CB * CB;
    RCHK(h2d(ctx, Li, hi.data(), kb * kb * sizeof(double)));
    const int64_t r0 = k0 + kb, rn = n - r0;
    if (rn <= 0) continue;
    // panel: A[r0:, k0:k0+kb] <- A[r0:, k0:k0+kb] L_kk^-T
    RCHK(gemm(ctx, mk(rn, kb, kb, A + r0 * n + k0, n, false, Li, kb, true, tmp, kb)));
    MISC(k_copy2d(1, rn, kb, tmp, kb, 0, A + r0 * n + k0, n, 0, false, ctx->stream));
    // trailing: A[r0:, r0:] -= panel panel^T
    RCHK(gemm(ctx, mk(rn, rn, kb, A + r0 * n + k0, n, false, A + r0 * n + k0, n, true, A + r0 * n + r0, n, -1.0, 1.0)));
  }
  return THC_OK;
}

// Solves L X = B (forward) or L^T X = B (backward) for X (n x m, row-major, in place in B).
int trsm(thc_ctx* ctx, const double* A, int64_t n, const double* Linv, double* B, int64_t m, bool backward,
         double* tmp) {
  const int64_t nblk = (n + CB - 1) / CB;
  for (int64_t bi = 0; bi < nblk; ++bi) {
    const int64_t b = backward ? nblk - 1 - bi : bi;
    const int64_t k0 = b * CB, kb = std::min(CB, n - k0);
    const double* Li = Linv + b * CB * CB;
    if (!backward) {
      if (k0 > 0)  // B_k -= L[k, :k0] X[:k0]
        RCHK(gemm(ctx, mk(kb, m, k0, A + k0 * n, n, false, B, m, false, B + k0 * m, m, -1.0, 1.0)));
      RCHK(gemm(ctx, mk(kb, m, kb, Li, kb, false, B + k0 * m, m, false, tmp, m)));
    } else {
      const int64_t r0 = k0 + kb;
      if (r0 < n)  // B_k -= L[r0:, k]^T X[r0:]
        RCHK(gemm(ctx, mk(kb, m, n - r0, A + r0 * n + k0, n, true, B + r0 * m, m, false, B + k0 * m, m, -1.0, 1.0)));
      RCHK(gemm(ctx, mk(kb, m, kb, Li, kb, true, B + k0 * m, m, false, tmp, m)));
    }
    MISC(k_copy2d(1, kb, m, tmp, m, 0, B + k0 * m, m, 0, false, ctx->stream));
  }
  return THC_OK;
}

int check_finite_host(thc_ctx* ctx, const double* x, size_t n, const char* what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) {
      ctx->err = std::string("non-finite value in ") + what;
      return THC_ENUMERIC;
    }
  return THC_OK;
}

// ---------------------------------------------------------------------------------------
// Working-memory plan.  Every device buffer of a context is a piece of one arena (one
// allocation, or the caller's workspace): the persistent buffers (factors, state, DIIS, the
// fused pass's block buffers, S and R of Alg. 7), the Alg. 6 region (the H block, its E, F, G
// grid-point chunk and the C, D operands), which the set-up also uses as its scratch before the
// first residual, and the chunk buffers of Alg. 7.  The plan picks the H block Xb (multiple of
// 64), the grid-point chunk Ic and the Alg. 7 row chunk X7 so the arena fits the budget: Ic near
// 256 or more (each chunk reads and writes the H block once: H traffic per residual is
// 16 P Pp^2 Q / Ic bytes, independent of Xb), then the largest Xb (each H block recomputes the
// G chunks, the paper's redundancy).
constexpr double MEM_CAP = 270.0e9;   // at most this much device memory without a workspace
constexpr size_t ALIGN_D = 32;       // buffers start on 256-byte boundaries

struct BufSpec {
  double** p;
  size_t n;  // doubles
};

size_t aligned(size_t n) { return (std::max<size_t>(n, 1) + ALIGN_D - 1) / ALIGN_D * ALIGN_D; }

double list_bytes(const std::vector<BufSpec>& l) {
  double b = 0.0;
  for (const auto& a : l) b += 8.0 * (double)aligned(a.n);
  return b;
}

std::vector<BufSpec> persistent_list(thc_ctx* ctx) {
  const int64_t o = ctx->o, v = ctx->v, n = ctx->n, nL = ctx->nL, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const int64_t PP = P * P, nb = ctx->nb, dm = ctx->opt.diis_max;
  const int64_t nlvv = ctx->lvv_resident ? nL : nb;
  return {
      {&ctx->Loo, (size_t)(nL * o * o)}, {&ctx->Lov, (size_t)(nL * ov)}, {&ctx->Lvv, (size_t)(nlvv * v * v)},
      {&ctx->eps, (size_t)n}, {&ctx->Yo, (size_t)(o * P)}, {&ctx->Yv, (size_t)(v * P)},
      {&ctx->xo, (size_t)(o * Q)}, {&ctx->xv, (size_t)(v * Q)}, {&ctx->Go, (size_t)PP}, {&ctx->Gv, (size_t)PP},
      {&ctx->S, (size_t)PP}, {&ctx->z, (size_t)(Q * Q)}, {&ctx->Bq, (size_t)(Q * ov)}, {&ctx->Bkr, (size_t)(ov * P)},
      {&ctx->W, (size_t)PP}, {&ctx->e, (size_t)P},
      {&ctx->Th, (size_t)PP}, {&ctx->Th0, (size_t)PP}, {&ctx->t1, (size_t)ov}, {&ctx->Zs, (size_t)PP},
      {&ctx->delta, (size_t)P},
      {&ctx->dvec, (size_t)(std::max<int64_t>(dm, 1) * (PP + ov))}, {&ctx->derr, (size_t)(std::max<int64_t>(dm, 1) * (PP + ov))},
      {&ctx->dT, (size_t)(PP + ov)},
      {&ctx->sig, (size_t)PP}, {&ctx->sig1, (size_t)ov}, {&ctx->sigh, (size_t)PP}, {&ctx->scal, 64},
      // fused pass
      {&ctx->Lhoo, (size_t)(nb * o * o)}, {&ctx->Lhvo, (size_t)(nb * v * o)}, {&ctx->tmpoo, (size_t)(nb * o * o)},
      {&ctx->tmpooT, (size_t)(nb * o * o)}, {&ctx->Pv, (size_t)(nb * v * o)}, {&ctx->PvT, (size_t)(nb * v * o)},
      {&ctx->LovYv, (size_t)(nb * o * P)}, {&ctx->Wv, (size_t)(nb * v * P)}, {&ctx->Bvv, (size_t)(nb * PP)},
      {&ctx->Woo, (size_t)(nb * o * P)}, {&ctx->Boo, (size_t)(nb * PP)}, {&ctx->Ccat, (size_t)(nb * PP)},
      {&ctx->Dcat, (size_t)(nb * PP)}, {&ctx->Wvo, (size_t)(nb * o * P)}, {&ctx->Y1, (size_t)(nb * o * P)},
      {&ctx->Gm, (size_t)(nb * ov)}, {&ctx->GY, (size_t)(nb * o * P)}, {&ctx->TA, (size_t)(P * nb)},
      {&ctx->tmpov, (size_t)(nb * std::max(std::max(ov, v * v), o * o))},
      {&ctx->sig28, (size_t)(ctx->KS * PP)}, {&ctx->C3, (size_t)PP}, {&ctx->Abar, (size_t)(P * nL)},
      {&ctx->At, (size_t)(P * nL)}, {&ctx->Hh, (size_t)(P * nL)}, {&ctx->xioo, (size_t)(o * o)},
      {&ctx->xivv, (size_t)(v * v)}, {&ctx->s38, (size_t)ov}, {&ctx->dvecA, (size_t)nL}, {&ctx->trK, (size_t)nL},
      {&ctx->ej, (size_t)nL}, {&ctx->ek, (size_t)(nL * 64)}, {&ctx->Fin, (size_t)(n * n)}, {&ctx->Fh, (size_t)(n * n)},
      {&ctx->Jov, (size_t)ov}, {&ctx->Jvo, (size_t)ov},
      // assembly
      {&ctx->ST, (size_t)PP}, {&ctx->Dt, (size_t)(P * nL)}, {&ctx->K29, (size_t)(P * nL)}, {&ctx->Qm, (size_t)PP},
      {&ctx->ot, (size_t)PP}, {&ctx->vt, (size_t)PP}, {&ctx->E9, (size_t)PP}, {&ctx->tmpoP, (size_t)(o * P)},
      {&ctx->tmpvP, (size_t)(v * P)}, {&ctx->Fxoo, (size_t)(o * o)}, {&ctx->Fxvv, (size_t)(v * v)},
      {&ctx->Tf, (size_t)P}, {&ctx->fd, (size_t)P},
      // Alg. 7 quantities needed for every X
      {&ctx->S7, (size_t)(P * ov)}, {&ctx->R7, (size_t)(P * ov)}, {&ctx->Cx, (size_t)(P * Q)}, {&ctx->Dx, (size_t)(P * Q)},
      {&ctx->gws, (size_t)GEMM_WS},
  };
}

// Alg. 6 region for an H block of Xb ranks and grid-point chunks of Ic points.  The mixed path's
// FP32 E, F live in the first half of the FP64 E, F buffers: a residual uses one precision or the
// other, and each writes every element (padding included) that its H-kernel reads.
std::vector<BufSpec> region6_list(thc_ctx* ctx) {
  const int64_t o = ctx->o, v = ctx->v, P = ctx->P, Pp = ctx->Pp, ov = ctx->ov, Xb = ctx->Xb, Ic = ctx->Ic;
  std::vector<BufSpec> l = {
      {&ctx->C6, (size_t)(o * Xb * Pp)}, {&ctx->D6, (size_t)(v * Xb * Pp)}, {&ctx->Ec, (size_t)(Ic * Xb * Pp)},
      {&ctx->Fc, (size_t)(Ic * Xb * Pp)}, {&ctx->Gc, (size_t)(Ic * Pp * Pp)}, {&ctx->GYc, (size_t)(Ic * o * P)},
      {&ctx->Hb, (size_t)(Xb * Pp * Pp)}, {&ctx->R1, (size_t)(Xb * Pp * o)}, {&ctx->I6, (size_t)(Xb * ov)}};
  return l;
}

std::vector<BufSpec> alg7_list(thc_ctx* ctx) {
  const int64_t o = ctx->o, P = ctx->P, Q = ctx->Q, ov = ctx->ov, X7 = ctx->X7;
  const bool fused = exch_supported(o) && !(ctx->opt.flags & THC_FLAG_UNFUSED_EXCHANGE);
  return {{&ctx->U7, (size_t)(X7 * o * P)}, {&ctx->Rx, (size_t)(X7 * o * Q)}, {&ctx->Sx, (size_t)(X7 * o * Q)},
          {&ctx->F7, (size_t)(fused ? 1 : ctx->Xc * Q * Q)}, {&ctx->Gt, (size_t)(X7 * o * Q)},
          {&ctx->Gts, (size_t)(X7 * o * Q)}, {&ctx->G7, (size_t)(X7 * ov)}, {&ctx->G7s, (size_t)(X7 * ov)}};
}

// Doubles of device scratch the set-up (thc_build_factors) holds at once.
size_t setup_doubles(const thc_ctx* ctx) {
  const int64_t o = ctx->o, nL = ctx->nL, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const int64_t CBn = (std::max(Q, P) + CB - 1) / CB;
  const int64_t rc0 = std::max<int64_t>(1, std::min<int64_t>(ov, (int64_t)(1.0e9 / (8.0 * ov))));
  size_t d = 0;
  for (int64_t c : {Q * Q, Q * Q, CBn * CB * CB, Q * nL, std::min<int64_t>(nL, 256) * o * Q,
                    std::max(Q, P) * std::max<int64_t>(std::max(nL, P), CB), CB * std::max(std::max(nL, P), Q),
                    P * P, P * P, P * P, rc0 * ov, rc0 * P})
    d += aligned((size_t)c);
  if (ctx->synth) d += aligned((size_t)(nL * nL)) + 2 * aligned((size_t)nL);  // the gamma rule
  return d;
}

// Tiles of the H-kernel table (X tile, Y block, Z block >= Y block, Z slice) and its length with
// the empty slots that complete the last generation.
void tile_counts(int64_t Pp, int64_t Xb, int64_t slots, int64_t* tiles, int64_t* entries) {
  const int64_t nB = Pp / 16, nX = Xb / 64;
  int64_t lin = 0;
  for (int64_t yb = 0; yb < nB; ++yb) lin += (nB - yb) * 2;
  lin *= nX;
  const int64_t runs = (lin + slots - 1) / slots;
  *tiles = lin;
  *entries = ((runs + 7) / 8) * 8 * slots;
}

size_t tile_table_doubles(int64_t Pp, int64_t Xb, int64_t slots) {
  int64_t t = 0, e = 0;
  tile_counts(Pp, Xb, slots, &t, &e);
  return aligned((size_t)((e + 1) / 2));
}

// Flops of the quadratic ladder and exchange terms (Eq. 32 + 33) by the O(N^5) Algorithms 4 and 5
// (every step a matrix product: per (i, j) pair of Alg. 4 and (j, a) pair of Alg. 5, the
// amplitudes, their Q x Q ERI transform, back, and the projection of the dense residual), and an
// estimate of their time against Alg. 6 at the measured rates (FP64 MFMA products ~45 TFLOP/s,
// the H-kernel ~26 TFLOP/s issued).
double quintic_flops(int64_t o, int64_t v, int64_t P, int64_t Q) {
  const double O = (double)o, V = (double)v, PP = (double)P, QQ = (double)Q, ov = O * V;
  const double a4 = O * O * (2 * V * V * PP + 2 * V * V * QQ + 2 * QQ * QQ * V + 2 * O * QQ * QQ + 2 * O * O * QQ +
                             2 * O * O * PP + 2 * O * PP * PP + 2 * V * PP * PP + 2 * V * V * PP);
  const double a5 = ov * (2 * ov * PP + 2 * ov * QQ + 2 * QQ * QQ * O + 2 * QQ * QQ * V + 2 * O * QQ * V + 2 * ov * PP +
                          2 * V * PP * PP + 2 * O * PP * PP + 2 * ov * PP);
  return a4 + a5 + 2 * O * PP * PP * V + 2 * ov * ov * PP + 2 * ov * PP * PP;
}

bool prefer_quintic(int64_t o, int64_t v, int64_t P, int64_t Q) {
  const double Pd = (double)P, Qd = (double)Q, od = (double)o, vd = (double)v;
  const double t6 = 3.5 * Qd * Pd * Pd * Pd / 26.0e12 +
                    (2 * (od + vd) * Pd * Pd * Qd + 2 * Qd * (od * vd * Pd + od * Pd * Pd) + 2 * vd * Pd * Pd * Pd) / 45.0e12;
  return quintic_flops(o, v, P, Q) / 45.0e12 < t6;
}

std::vector<BufSpec> quintic_list(thc_ctx* ctx) {
  const int64_t o = ctx->o, v = ctx->v, P = ctx->P, Q = ctx->Q, ov = ctx->ov, w = std::max(o, v), n = ctx->nq;
  return {{&ctx->Wq, (size_t)(o * P * v)},          {&ctx->qT1, (size_t)(ov * P)},
          {&ctx->qR, (size_t)(ov * ctx->jq * v)},    {&ctx->qC, (size_t)(n * std::max(v * v, ov))},
          {&ctx->qD1, (size_t)(n * w * Q)},          {&ctx->qE, (size_t)(n * Q * Q)},
          {&ctx->qF1, (size_t)(n * w * Q)},          {&ctx->qF, (size_t)(n * std::max(o * o, ov))},
          {&ctx->qG1, (size_t)(n * w * P)},          {&ctx->qG, (size_t)(n * P * P)},
          {&ctx->qI1, (size_t)(n * w * P)}};
}

// Picks the blocking (nb, KS, Xb, Ic, X7, the residency of the vv block) for a budget of device
// bytes and fills ctx->plan_bytes; THC_ENOMEM if even the smallest blocking does not fit.
int choose_plan(thc_ctx* ctx, double budget, int64_t slots) {
  const int64_t o = ctx->o, v = ctx->v, nL = ctx->nL, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const int64_t Pp = ctx->Pp = ((P + 15) / 16) * 16;  // Y, Z ranks of H padded to its 16-wide blocks
  const int64_t P64 = ((P + 63) / 64) * 64;           // X ranks padded to its 64-lane tiles
  const thc_options& op = ctx->opt;
  // fused-pass block: four nb x P^2 panels within ~4 GB
  int64_t nb = op.a_block > 0 ? op.a_block : std::max<int64_t>(1, std::min<int64_t>(64, (int64_t)(4.0e9 / (32.0 * P * P))));
  ctx->nb = nb = std::min(nb, nL);
  // split of the N_L P-deep sum of Alg. 1: at most 512 workgroups of 128 x 128 tiles (one round
  // at two per CU), counting the tiles on and above the diagonal (the product is symmetric)
  const int64_t nt128 = (P + 127) / 128, t128 = nt128 * (nt128 + 1) / 2;
  ctx->KS = std::max<int64_t>(1, std::min<int64_t>(16, 512 / t128));
  {
    Gemm g;  // the first block's sum_A C^A T C^A^T, as residual_impl issues it
    g.M = g.N = P;
    g.K = nb * P;
    g.ksplit = (int)ctx->KS;
    g.upper = true;
    ctx->alg1_tile = gemm_tile_edge_split(g);
  }
  // the vv Cholesky block: held (caller inputs always); synthetic inputs regenerate it block by
  // block in the fused pass when asked or when it would take more than 40% of the budget
  ctx->lvv_resident = !ctx->synth || (!(op.flags & THC_FLAG_STREAM_LVV) && 8.0 * (double)nL * v * v < 0.4 * budget);
  int64_t Xc = op.x_chunk;
  if (Xc <= 0) Xc = std::max<int64_t>(1, (int64_t)(2.0e9 / (8.0 * (double)Q * Q)));
  ctx->Xc = std::min(Xc, P);
  // Alg. 7 row chunk: every row when the chunked intermediates (U, Rx, Sx, Gt, Gt~, G, G~:
  // o P + 4 o Q + 2 o v per row) fit in min(24 GB, a tenth of the budget)
  int64_t X7 = op.x7_chunk;
  const double per7 = 8.0 * (double)(o * P + 4 * o * Q + 2 * ov);
  if (X7 <= 0) X7 = std::max<int64_t>(1, (int64_t)(std::min(24.0e9, 0.1 * budget) / per7));
  ctx->X7 = std::min(X7, P);
  const double pers = list_bytes(persistent_list(ctx));
  const double a7 = list_bytes(alg7_list(ctx));
  const double setup = 8.0 * (double)setup_doubles(ctx);
  // Eq. 32 + 33 by Alg. 4 and 5 (asked for, or estimated faster) instead of Alg. 6
  ctx->quintic = (op.flags & THC_FLAG_QUINTIC) ||
                 (!(op.flags & THC_FLAG_QUARTIC) && prefer_quintic(o, v, P, Q));
  if (ctx->quintic) {
    ctx->Xb = std::min<int64_t>(64, P64);  // no H block; the tile table stays minimal
    ctx->Ic = 1;
    const double fixedq = 8.0 * ((double)o * P * v + (double)ov * P);
    const double left = budget - pers - a7 - fixedq;
    const int64_t w = std::max(o, v);
    const double per_pair = 8.0 * (double)(aligned((size_t)std::max(v * v, ov)) + 2 * aligned((size_t)(w * Q)) +
                                           aligned((size_t)(Q * Q)) + aligned((size_t)std::max(o * o, ov)) +
                                           2 * aligned((size_t)(w * P)) + aligned((size_t)(P * P)));
    // the dense residual for all j when it takes at most half of what is left, else by chunks of j
    int64_t jq = o;
    if (8.0 * (double)ov * ov > 0.5 * left) jq = std::max<int64_t>(1, (int64_t)(0.5 * left / (8.0 * (double)ov * v)));
    ctx->jq = std::min(op.q_jchunk > 0 ? op.q_jchunk : jq, o);
    const double rbytes = 8.0 * (double)ov * ctx->jq * v;
    ctx->nq = std::min<int64_t>(w, (int64_t)((left - rbytes) / per_pair));
    if (op.q_pairs > 0) ctx->nq = std::min(ctx->nq, op.q_pairs);
    if (ctx->nq < 1 || budget - pers - a7 < setup) {
      ctx->err = "the working memory of Alg. 4 and 5 does not fit the budget";
      return THC_ENOMEM;
    }
    return THC_OK;
  }
  // H block and grid-point chunk
  auto fixed6 = [&](int64_t Xb) { return 8.0 * (double)Xb * ((double)Pp * (o + v + Pp + o) + (double)ov); };
  auto per_i = [&](int64_t Xb) {
    return 8.0 * (2.0 * (double)Xb * Pp + (double)Pp * Pp + (double)o * P);
  };
  if (op.x_block > 0 && (op.x_block % 64 != 0 || op.x_block > P64)) {
    ctx->err = "x_block must be a multiple of 64 and at most the rank rounded up to 64";
    return THC_EINVAL;
  }
  const int64_t ic_min = op.i_chunk > 0 ? std::min(op.i_chunk, Q) : std::min<int64_t>(Q, 256);
  int64_t Xb = 0;
  double rem = 0.0;
  for (int64_t xb = op.x_block > 0 ? op.x_block : P64; xb >= 64; xb -= 64) {
    // the FP32 kernel's table (mixed precision) has half as many tiles: at most as many entries
    const double tiles = 8.0 * (double)tile_table_doubles(Pp, xb, slots) * (op.precision >= 1 ? 2.0 : 1.0);
    rem = budget - pers - a7 - tiles - fixed6(xb);
    const double r6 = fixed6(xb) + per_i(xb) * (double)ic_min;
    if (rem >= per_i(xb) * (double)ic_min && rem + r6 - std::max(r6, setup) >= 0.0) {
      Xb = xb;
      break;
    }
    if (op.x_block > 0) break;
  }
  if (Xb == 0) {
    char buf[300];
    snprintf(buf, sizeof buf,
             "the working memory does not fit %.1f GB: %.1f GB persistent (factors, state, fused-pass blocks), "
             "%.1f GB Alg. 7 chunks, and an H block of 64 ranks with %lld grid points needs %.1f GB more",
             budget / 1e9, pers / 1e9, a7 / 1e9, (long long)ic_min, (fixed6(64) + per_i(64) * ic_min) / 1e9);
    ctx->err = buf;
    return THC_ENOMEM;
  }
  ctx->Xb = Xb;
  int64_t Ic = op.i_chunk;
  if (Ic <= 0) Ic = std::max<int64_t>(1, (int64_t)(std::min(rem, std::max(16.0e9, 256.0 * per_i(Xb))) / per_i(Xb)));
  ctx->Ic = std::min(Ic, Q);
  return THC_OK;
}

// The plan for the context's budget (its workspace, else the device's free memory up to
// MEM_CAP), then the arena and every buffer in it.
int plan_and_alloc(thc_ctx* ctx) {
  ctx->hslots = h_slots_per_xcd();
  if (ctx->hslots < 1) { ctx->err = "cannot query the device for the H-kernel launch"; return THC_EDEVICE; }
  double budget = (double)ctx->ws_bytes;
  if (!ctx->ws) {
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) { ctx->err = "hipMemGetInfo failed"; return THC_EDEVICE; }
    budget = std::min(MEM_CAP, (double)freeb - 2.0e9);
  }
  RCHK(choose_plan(ctx, budget, ctx->hslots));
  const std::vector<uint32_t> tiles = h_tiles(ctx->Pp, ctx->Xb, ctx->hslots);
  std::vector<uint32_t> tiles32;
  if (ctx->opt.precision >= 1 && !ctx->quintic) {
    ctx->hslots32 = h32_slots_per_xcd();
    if (ctx->hslots32 < 1) { ctx->err = "cannot query the device for the H-kernel launch"; return THC_EDEVICE; }
    tiles32 = h32_tiles(ctx->Pp, ctx->Xb, ctx->hslots32);
  }
  double* tb = nullptr;
  std::vector<BufSpec> pers = persistent_list(ctx);
  pers.push_back({&tb, (tiles.size() + tiles32.size() + 1) / 2});
  const std::vector<BufSpec> r6 = ctx->quintic ? quintic_list(ctx) : region6_list(ctx), a7 = alg7_list(ctx);
  size_t np = 0, n6 = 0, n7 = 0;
  for (const auto& a : pers) np += aligned(a.n);
  for (const auto& a : r6) n6 += aligned(a.n);
  for (const auto& a : a7) n7 += aligned(a.n);
  const size_t nsetup = setup_doubles(ctx);
  const size_t total = np + std::max(n6, nsetup) + n7;
  if (ctx->ws) {
    if (8.0 * (double)total > (double)ctx->ws_bytes) { ctx->err = "workspace too small for the plan"; return THC_ENOMEM; }
    ctx->arena = (double*)ctx->ws;
  } else {
    void* q = nullptr;
    if (hipMalloc(&q, total * sizeof(double)) != hipSuccess) {
      char buf[160];
      snprintf(buf, sizeof buf, "hipMalloc of the %.2f GB working memory failed", 8.0 * (double)total / 1e9);
      ctx->err = buf;
      (void)hipGetLastError();
      return THC_ENOMEM;
    }
    ctx->allocs.push_back(q);
    ctx->arena = (double*)q;
  }
  ctx->bytes = total * sizeof(double);
  double* at = ctx->arena;
  for (const auto& a : pers) { *a.p = at; at += aligned(a.n); }
  ctx->setup_scratch = at;  // the set-up's scratch overlays the Alg. 6 region
  ctx->setup_len = std::max(n6, nsetup);
  for (const auto& a : r6) { *a.p = at; at += aligned(a.n); }
  at = ctx->setup_scratch + std::max(n6, nsetup);
  for (const auto& a : a7) { *a.p = at; at += aligned(a.n); }
  ctx->Ec32 = ctx->opt.precision >= 1 && !ctx->quintic ? reinterpret_cast<float*>(ctx->Ec) : nullptr;
  ctx->Fc32 = ctx->opt.precision >= 1 && !ctx->quintic ? reinterpret_cast<float*>(ctx->Fc) : nullptr;
  ctx->htiles = reinterpret_cast<uint32_t*>(tb);
  ctx->nhtiles = (int64_t)tiles.size();
  ctx->hfilled = 0;
  for (uint32_t t : tiles) ctx->hfilled += (t & 0x80000000u) ? 0 : 1;
  RCHK(h2d(ctx, ctx->htiles, tiles.data(), tiles.size() * sizeof(uint32_t)));
  if (!tiles32.empty()) {
    ctx->htiles32 = ctx->htiles + tiles.size();
    ctx->nhtiles32 = (int64_t)tiles32.size();
    RCHK(h2d(ctx, ctx->htiles32, tiles32.data(), tiles32.size() * sizeof(uint32_t)));
    // FP32 G in the FP64 G buffer (a residual uses one or the other)
    ctx->G32 = reinterpret_cast<float*>(ctx->Gc);
  }
  ctx->diisB.assign((size_t)std::max<int64_t>(ctx->opt.diis_max, 1) * std::max<int64_t>(ctx->opt.diis_max, 1), 0.0);
  return THC_OK;
}

// The Alg. 6 operands whose padding must stay zero, cleared once the set-up no longer uses the
// region as scratch.
int clear_region6(thc_ctx* ctx) {
  if (ctx->quintic) return THC_OK;  // Alg. 4 and 5 need no zero padding
  const int64_t o = ctx->o, v = ctx->v, Pp = ctx->Pp, Xb = ctx->Xb, Ic = ctx->Ic;
  RCHK(zero(ctx, ctx->C6, o * Xb * Pp));
  RCHK(zero(ctx, ctx->D6, v * Xb * Pp));
  RCHK(zero(ctx, ctx->Gc, Ic * Pp * Pp));
  RCHK(zero(ctx, ctx->Hb, Xb * Pp * Pp));
  RCHK(zero(ctx, ctx->Ec, Ic * Xb * Pp));
  RCHK(zero(ctx, ctx->Fc, Ic * Xb * Pp));  // also the FP32 copies, which share this memory
  return THC_OK;
}

// With THC_FLAG_PROGRESS: waits for the stream and prints one line to stderr (long residuals at
// the largest workloads report each finished block of the paper's loops).
int progress(thc_ctx* ctx, const char* what, int64_t done, int64_t total) {
  if (!(ctx->opt.flags & THC_FLAG_PROGRESS)) return THC_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  fprintf(stderr, "thc: %s %lld/%lld\n", what, (long long)done, (long long)total);
  fflush(stderr);
  return THC_OK;
}

// Copies one scalar region of ctx->scal to the host.
int read_scalars(thc_ctx* ctx, double* h, int count) {
  RCHK(d2h(ctx, h, ctx->scal, count * sizeof(double)));
  return THC_OK;
}

// ---------------------------------------------------------------------------------------
// Eq. 32 and 33 by Alg. 4 and 5: sigma += B^T R B with R_(ia)(jb) the dense quadratic ladder
// (Alg. 4: sum_kl X_ij^kl t_kl^ab, X_ij^kl = sum_cd t_ij^cd (kc|ld)) and exchange (Alg. 5:
// sum_kcld t_ik^cb t_lj^ad (lc|kd)) terms, formed pair by pair as matrix products in batches of
// pairs, with the THC form of (ia|jb); R is held for a chunk of occupied j at a time.
int quintic_terms(thc_ctx* ctx, const double* T) {
  const int64_t o = ctx->o, v = ctx->v, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const double *Yo = ctx->Yo, *Yv = ctx->Yv, *xo = ctx->xo, *xv = ctx->xv, *z = ctx->z;
  // W_j[Z][d] = sum_Z' T[Z][Z'] y_j^Z' y_d^Z'  (the right half of t_.j^.d for every j)
  {
    Gemm g = batched(mk(P, v, P, T, P, false, Yv, P, true, ctx->Wq, v), o, 0, 0, P * v);
    g.kscaleB = Yo; g.ksB = 1; g.sksB = P;
    RCHK(gemm(ctx, g));
  }
  const int64_t nq = ctx->nq, jq = ctx->jq, ldR = jq * v;
  for (int64_t j0 = 0; j0 < o; j0 += jq) {
    const int64_t jc = std::min(jq, o - j0);
    // Alg. 4: pairs (i, j), a batch of j for each i
    for (int64_t i = 0; i < o; ++i) {
      for (int64_t b0 = 0; b0 < jc; b0 += nq) {
        const int64_t nb = std::min(nq, jc - b0), j = j0 + b0;
        // C[c][d] = t_ij^cd = sum_Z y_c^Z y_i^Z W_j[Z][d]
        Gemm g = batched(mk(v, v, P, Yv, P, false, ctx->Wq + j * P * v, v, false, ctx->qC, v), nb, 0, P * v, v * v);
        g.kscaleA = Yo + i * P; g.ksA = 1;
        RCHK(gemm(ctx, g));
        // E = z o (xv^T C xv);  F = xo E xo^T = X_ij^kl
        RCHK(gemm(ctx, batched(mk(v, Q, v, ctx->qC, v, false, xv, Q, false, ctx->qD1, Q), nb, v * v, 0, v * Q)));
        Gemm ge = batched(mk(Q, Q, v, xv, Q, true, ctx->qD1, Q, false, ctx->qE, Q), nb, 0, v * Q, Q * Q);
        ge.hmul = z; ge.ldh = Q;
        RCHK(gemm(ctx, ge));
        RCHK(gemm(ctx, batched(mk(o, Q, Q, xo, Q, false, ctx->qE, Q, false, ctx->qF1, Q), nb, 0, Q * Q, o * Q)));
        RCHK(gemm(ctx, batched(mk(o, o, Q, ctx->qF1, Q, false, xo, Q, true, ctx->qF, o), nb, o * Q, 0, o * o)));
        // H = T o (Yo^T F Yo);  R_ij^ab = (Yv H Yv^T)_ab = sum_kl X_ij^kl t_kl^ab
        RCHK(gemm(ctx, batched(mk(o, P, o, ctx->qF, o, false, Yo, P, false, ctx->qG1, P), nb, o * o, 0, o * P)));
        Gemm gh = batched(mk(P, P, o, Yo, P, true, ctx->qG1, P, false, ctx->qG, P), nb, 0, o * P, P * P);
        gh.hmul = T; gh.ldh = P;
        RCHK(gemm(ctx, gh));
        RCHK(gemm(ctx, batched(mk(v, P, P, Yv, P, false, ctx->qG, P, false, ctx->qI1, P), nb, 0, P * P, v * P)));
        RCHK(gemm(ctx, batched(mk(v, v, P, ctx->qI1, P, false, Yv, P, true, ctx->qR + i * v * ldR + b0 * v, ldR),
                               nb, v * P, 0, v)));
      }
    }
    // Alg. 5: pairs (j, a), a batch of a for each j; adds sum_kcld t_ik^cb t_lj^ad (lc|kd) to R
    for (int64_t jj = 0; jj < jc; ++jj) {
      const int64_t j = j0 + jj;
      for (int64_t a0 = 0; a0 < v; a0 += nq) {
        const int64_t na = std::min(nq, v - a0);
        // C[l][d] = t_lj^ad = sum_Z y_l^Z y_a^Z W_j[Z][d]
        Gemm g = batched(mk(o, v, P, Yo, P, false, ctx->Wq + j * P * v, v, false, ctx->qC, v), na, 0, 0, ov);
        g.kscaleA = Yv + a0 * P; g.ksA = 1; g.sksA = P;
        RCHK(gemm(ctx, g));
        // E = z o (xo^T C xv);  F[k][c] = sum_J xo[k][J] sum_I E[I][J] xv[c][I]
        RCHK(gemm(ctx, batched(mk(o, Q, v, ctx->qC, v, false, xv, Q, false, ctx->qD1, Q), na, ov, 0, o * Q)));
        Gemm ge = batched(mk(Q, Q, o, xo, Q, true, ctx->qD1, Q, false, ctx->qE, Q), na, 0, o * Q, Q * Q);
        ge.hmul = z; ge.ldh = Q;
        RCHK(gemm(ctx, ge));
        RCHK(gemm(ctx, batched(mk(Q, v, Q, ctx->qE, Q, true, xv, Q, true, ctx->qF1, v), na, Q * Q, 0, Q * v)));
        RCHK(gemm(ctx, batched(mk(o, v, Q, xo, Q, false, ctx->qF1, v, false, ctx->qF, v), na, 0, Q * v, ov)));
        // H = T o (Yv^T F^T Yo);  R_ij^ab += (Yo H Yv^T)_ib
        RCHK(gemm(ctx, batched(mk(v, P, o, ctx->qF, v, true, Yo, P, false, ctx->qG1, P), na, ov, 0, v * P)));
        Gemm gh = batched(mk(P, P, v, Yv, P, true, ctx->qG1, P, false, ctx->qG, P), na, 0, v * P, P * P);
        gh.hmul = T; gh.ldh = P;
        RCHK(gemm(ctx, gh));
        RCHK(gemm(ctx, batched(mk(o, P, P, Yo, P, false, ctx->qG, P, false, ctx->qI1, P), na, 0, P * P, o * P)));
        RCHK(gemm(ctx, batched(mk(o, v, P, ctx->qI1, P, false, Yv, P, true, ctx->qR + a0 * ldR + jj * v, v * ldR,
                                  1.0, 1.0), na, o * P, 0, ldR)));
      }
    }
    // sigma += B^T R B over the chunk's columns (jb)
    RCHK(gemm(ctx, mk(ov, P, jc * v, ctx->qR, ldR, false, ctx->Bkr + j0 * v * P, P, false, ctx->qT1, P)));
    RCHK(gemm(ctx, mk(P, P, ov, ctx->Bkr, P, true, ctx->qT1, P, false, ctx->sig, P, 1.0, 1.0)));
    RCHK(progress(ctx, "Alg. 4 and 5 occupied chunks", j0 / jq + 1, (o + jq - 1) / jq));
  }
  return THC_OK;
}

// ---------------------------------------------------------------------------------------
// The residual (and the energy of the same amplitudes).  T: raw core (device, P x P);
// t1: singles (device, may be null).  Results in ctx->sig (P x P), ctx->sig1 (o x v) and the
// energy partial sums in ctx->scal[0..3] (E_J, E_K, singles: 2 sum d_A^2, sum tr K_A^2).
int residual_impl(thc_ctx* ctx, const double* T, const double* t1, uint32_t mask) {
  Scope whole(ctx, "residual");
  MixedScope precision(ctx);
  hipStream_t s = ctx->stream;
  const int64_t o = ctx->o, v = ctx->v, n = ctx->n, nL = ctx->nL, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const int64_t PP = P * P, Pp = ctx->Pp;
  const bool sres = ctx->opt.singles != 0;    // singles residual wanted
  const bool singles = sres && t1 != nullptr;  // T1 dressing needed (t1 given)
  const double *Yo = ctx->Yo, *Yv = ctx->Yv, *xo = ctx->xo, *xv = ctx->xv;

  RCHK(zero(ctx, ctx->sig, PP));
  RCHK(zero(ctx, ctx->sig1, ov));
  RCHK(zero(ctx, ctx->sig28, ctx->KS * PP));
  RCHK(zero(ctx, ctx->C3, PP));
  RCHK(zero(ctx, ctx->xioo, o * o));
  RCHK(zero(ctx, ctx->xivv, v * v));
  RCHK(zero(ctx, ctx->s38, ov));
  RCHK(zero(ctx, ctx->Fin, n * n));
  RCHK(zero(ctx, ctx->dvecA, nL));
  RCHK(zero(ctx, ctx->trK, nL));

  // ---------------- fused pass over blocks of Cholesky vectors (Alg. 1, 2, 3, 8) -------------
  ctx->section = "gemm@fused";
  ctx->chain = 0;
  for (int64_t A0 = 0; A0 < nL; A0 += ctx->nb) {
    const int64_t nb = std::min(ctx->nb, nL - A0);
    const double* Loo = ctx->Loo + A0 * o * o;
    const double* Lov = ctx->Lov + A0 * ov;
    if (A0 > 0 && (A0 / ctx->nb) % std::max<int64_t>(1, (nL / ctx->nb) / 8) == 0)
      RCHK(progress(ctx, "fused Cholesky pass, vectors", A0, nL));
    const double* Lvv = ctx->lvv_resident ? ctx->Lvv + A0 * v * v : ctx->Lvv;
    if (!ctx->lvv_resident)  // the block's vv Cholesky panels from the generator
      MISC(synth_chol_block(ctx->spec.seed, n, A0, nb, o, v, o, v, ctx->spec.decay, ctx->gamma, ctx->Lvv, s));
    const double* Lhoo = Loo;  // dressed blocks (Eq. 27); the undressed ones in CCD mode
    if (singles) {
      // tmpoo[A] = Lov t1^T (o x o), also in the [i][A][k] layout for the Fock K-term
      RCHK(gemm(ctx, k64(batched(mk(o, o, v, Lov, v, false, t1, v, true, ctx->tmpoo, o), nb, ov, 0, o * o))));
      RCHK(gemm(ctx, k64(batched(mk(o, o, v, Lov, v, false, t1, v, true, ctx->tmpooT, nb * o), nb, ov, 0, o))));
      MISC(k_copy2d(1, nb * o, o, Loo, o, 0, ctx->Lhoo, o, 0, false, s));
      MISC(k_axpby(nb * o * o, 1.0, ctx->tmpoo, 1.0, ctx->Lhoo, s));
      Lhoo = ctx->Lhoo;
      MISC(k_trace_sq(nb, o, ctx->tmpoo, ctx->trK + A0, s));
      // d_A = sum_ia t_ia L_ia^A
      MISC(k_gemv(nb, ov, Lov, ov, t1, ctx->dvecA + A0, s));
      // Pv[A] = Lvv t1^T (v x o), in [A][a][k] and [a][A][k] layouts
      RCHK(gemm(ctx, k64(batched(mk(v, o, v, Lvv, v, false, t1, v, true, ctx->Pv, o), nb, v * v, 0, v * o))));
      RCHK(gemm(ctx, k64(batched(mk(v, o, v, Lvv, v, false, t1, v, true, ctx->PvT, nb * o), nb, v * v, 0, o))));
      // Lhvo[A] = Lov^T + Lvv t1^T - t1^T Lhoo
      MISC(k_copy2d(nb, v, o, Lov, v, ov, ctx->Lhvo, o, v * o, true, s));
      MISC(k_axpby(nb * v * o, 1.0, ctx->Pv, 1.0, ctx->Lhvo, s));
      RCHK(gemm(ctx, k64(batched(mk(v, o, o, t1, v, true, ctx->Lhoo, o, false, ctx->Lhvo, o, -1.0, 1.0), nb, 0, o * o, v * o))));
      // Fock: inner += 2 sum_A d_A L^A - sum_A (L^A[:, vir] t1^T) L^A[occ, :]
      MISC(k_wsum(nb, o * o, ctx->dvecA + A0, Loo, o * o, 2.0, ctx->Fin, s));  // oo block written densely below
      // (the block layout of Fin: [oo | ov | vo | vv] stored contiguously)
      MISC(k_wsum(nb, ov, ctx->dvecA + A0, Lov, ov, 2.0, ctx->Fin + o * o, s));
      MISC(k_wsum(nb, v * v, ctx->dvecA + A0, Lvv, v * v, 2.0, ctx->Fin + o * o + 2 * ov, s));
      RCHK(gemm(ctx, k64(mk(o, o, nb * o, ctx->tmpooT, nb * o, false, Loo, o, false, ctx->Fin, o, -1.0, 1.0))));
      RCHK(gemm(ctx, k64(mk(o, v, nb * o, ctx->tmpooT, nb * o, false, Lov, v, false, ctx->Fin + o * o, v, -1.0, 1.0))));
      RCHK(gemm(ctx, k64(mk(v, o, nb * o, ctx->PvT, nb * o, false, Loo, o, false, ctx->Fin + o * o + ov, o, -1.0, 1.0))));
      RCHK(gemm(ctx, k64(mk(v, v, nb * o, ctx->PvT, nb * o, false, Lov, v, false, ctx->Fin + o * o + 2 * ov, v, -1.0, 1.0))));
    }
    // LovYv[A] = Lov Yv (o x P)
    RCHK(gemm(ctx, k64(batched(mk(o, P, v, Lov, v, false, Yv, P, false, ctx->LovYv, P), nb, ov, 0, o * P))));
    // Wv[A] = L^vv Yv (v x P), dressed by - t1^T (Lov Yv)
    RCHK(gemm(ctx, batched(mk(v, P, v, Lvv, v, false, Yv, P, false, ctx->Wv, P), nb, v * v, 0, v * P)));
    if (singles)
      RCHK(gemm(ctx, batched(mk(v, P, o, t1, v, true, ctx->LovYv, P, false, ctx->Wv, P, -1.0, 1.0), nb, 0, o * P, v * P)));
    // Bvv[A] = Yv^T Wv[A];  Boo[A] = Yo^T (L^oo)^T Yo   (Alg. 1)
    RCHK(gemm(ctx, batched(mk(P, P, v, Yv, P, true, ctx->Wv, P, false, ctx->Bvv, P), nb, 0, v * P, PP)));
    RCHK(gemm(ctx, batched(mk(o, P, o, Lhoo, o, true, Yo, P, false, ctx->Woo, P), nb, o * o, 0, o * P)));
    RCHK(gemm(ctx, batched(mk(P, P, o, Yo, P, true, ctx->Woo, P, false, ctx->Boo, P), nb, 0, o * P, PP)));
    // C^A = Go o Bvv - Gv o Boo ([X][A][Y]); C3 += Boo o Bvv  (Alg. 1, Alg. 3)
    MISC(k_form_C(P, nb, ctx->Bvv, ctx->Boo, ctx->Go, ctx->Gv, ctx->Ccat, ctx->C3, s));
    if (mask & THC_TERM_EQ28) {
      // D^A = C^A T; sigma += sum_A D^A (C^A)^T  (Alg. 1), split over K
      RCHK(gemm(ctx, batched(mk(P, P, P, ctx->Ccat, nb * P, false, T, P, false, ctx->Dcat, nb * P), nb, P, 0, P)));
      // sum_A C^A T (C^A)^T is symmetric for a symmetric T (whether or not the T1-dressed C^A
      // are): only the tiles on and above the diagonal are computed; the reduction mirrors them
      Gemm g = mk(P, P, nb * P, ctx->Dcat, nb * P, false, ctx->Ccat, nb * P, true, ctx->sig28, P, 1.0, 1.0);
      g.ksplit = (int)ctx->KS;
      g.sSplit = PP;
      g.upper = true;
      RCHK(gemm(ctx, g));
    }
    // Abar^X_A = sum_ai y_a^X y_i^X L^_ai ; Atil^X_A = sum_ia y_i^X y_a^X L_ia  (Alg. 2)
    if (singles)
      RCHK(gemm(ctx, batched(mk(o, P, v, ctx->Lhvo, o, true, Yv, P, false, ctx->Wvo, P), nb, v * o, 0, o * P)));
    MISC(k_colsum_rowscaled(nb, o, P, Yo, singles ? ctx->Wvo : ctx->LovYv, o * P, ctx->Abar + A0, nL, s));
    MISC(k_colsum_rowscaled(nb, o, P, Yo, ctx->LovYv, o * P, ctx->At + A0, nL, s));
    // M^T[A] = (Lov Yv)^T Yo ; F = T o M^T ; exchange energy partials  (Alg. 2)
    RCHK(gemm(ctx, k64(batched(mk(P, P, o, ctx->LovYv, P, true, Yo, P, false, ctx->Boo, P), nb, o * P, 0, PP))));
    MISC(k_hadamard_energy(P, nb, T, ctx->Boo, ctx->Bvv, ctx->ek + A0 * 64, s));
    // G[A] = Yo F Yv^T (o x v); H^X_A = sum_ia y_i^X y_a^X G_ia  (Alg. 2)
    RCHK(gemm(ctx, batched(mk(o, P, P, Yo, P, false, ctx->Bvv, P, false, ctx->Y1, P), nb, 0, PP, o * P)));
    RCHK(gemm(ctx, batched(mk(o, v, P, ctx->Y1, P, false, Yv, P, true, ctx->Gm, v), nb, o * P, 0, ov)));
    RCHK(gemm(ctx, batched(mk(o, P, v, ctx->Gm, v, false, Yv, P, false, ctx->GY, P), nb, ov, 0, o * P)));
    MISC(k_colsum_rowscaled(nb, o, P, Yo, ctx->GY, o * P, ctx->Hh + A0, nL, s));
    // TA = T Atil (P x nb); Coulomb energy partials Atil^T T Atil
    RCHK(gemm(ctx, k64(mk(P, nb, P, T, P, false, ctx->At + A0, nL, false, ctx->TA, nb))));
    MISC(k_dot_cols(P, nb, ctx->At + A0, nL, ctx->TA, nb, ctx->ej + A0, s));
    // D8[A] = 2 Yo diag(T Atil_A) Yv^T - G[A]  (Alg. 8), in place of G
    {
      Gemm g = batched(mk(o, v, P, Yo, P, false, Yv, P, true, ctx->Gm, v, 2.0, -1.0), nb, 0, 0, ov);
      g.kscaleA = ctx->TA; g.ksA = nb; g.sksA = 1;
      RCHK(gemm(ctx, g));
    }
    // xi_oo += sum_A Lov D8^T ; xi_vv -= sum_A D8^T Lov  (Alg. 8)
    RCHK(gemm(ctx, batched(mk(o, o, v, Lov, v, false, ctx->Gm, v, true, ctx->tmpov, o), nb, ov, ov, o * o)));
    MISC(k_batch_sum(nb, o * o, ctx->tmpov, 1.0, ctx->xioo, s));
    RCHK(gemm(ctx, mk(v, v, nb * o, ctx->Gm, v, true, Lov, v, false, ctx->xivv, v, -1.0, 1.0)));
    if (sres) {
      // singles (Alg. 8, with the dressing folded into xi afterwards):
      // s38 += sum_A D8 Lvv - Loo D8
      RCHK(gemm(ctx, batched(mk(o, v, v, ctx->Gm, v, false, Lvv, v, false, ctx->tmpov, v), nb, ov, v * v, ov)));
      RCHK(gemm(ctx, batched(mk(o, v, o, Loo, o, false, ctx->Gm, v, false, ctx->tmpov, v, -1.0, 1.0), nb, o * o, ov, ov)));
      MISC(k_batch_sum(nb, ov, ctx->tmpov, 1.0, ctx->s38, s));
    }
  }
  RCHK(progress(ctx, "fused Cholesky pass done, vectors", nL, nL));
  // energy partial sums: scal[0] = sum_A Atil^T T Atil, scal[1] = exchange, scal[2] = sum d_A^2,
  // scal[3] = sum tr(K_A^2)
  MISC(k_sum(nL, ctx->ej, ctx->scal + 0, s));
  MISC(k_sum(nL * 64, ctx->ek, ctx->scal + 1, s));
  MISC(k_dot(nL, ctx->dvecA, ctx->dvecA, ctx->scal + 2, s));
  MISC(k_sum(nL, ctx->trK, ctx->scal + 3, s));

  // ---------------- Fock matrix, T1-transformed (Eq. 24-27) -----------------------------------
  ctx->section = "gemm@fock";
  ctx->chain = -1;
  ctx->mixed = false;  // the T1-transformed Fock matrix stays FP64
  double* Foo = ctx->Fh;
  double* Fov = ctx->Fh + o * o;
  double* Fvo = ctx->Fh + o * o + ov;
  double* Fvv = ctx->Fh + o * o + 2 * ov;
  {
    double* Ioo = ctx->Fin;
    double* Iov = ctx->Fin + o * o;
    double* Ivo = ctx->Fin + o * o + ov;
    double* Ivv = ctx->Fin + o * o + 2 * ov;
    MISC(k_set_diag(o, ctx->eps, Ioo, o, s));
    MISC(k_set_diag(v, ctx->eps + o, Ivv, v, s));
    if (singles) {
      // J part of the vo block: (2 sum_A d_A L_ov^A)^T (L symmetric)
      RCHK(zero(ctx, ctx->Jov, ov));
      MISC(k_wsum(nL, ov, ctx->dvecA, ctx->Lov, ov, 2.0, ctx->Jov, s));
      MISC(k_copy2d(1, v, o, ctx->Jov, v, 0, ctx->Jvo, o, 0, true, s));
      MISC(k_axpby(v * o, 1.0, ctx->Jvo, 1.0, Ivo, s));
      // F^ = (1 - tau) inner (1 + tau)
      MISC(k_copy2d(1, o, v, Iov, v, 0, Fov, v, 0, false, s));
      MISC(k_copy2d(1, o, o, Ioo, o, 0, Foo, o, 0, false, s));
      RCHK(gemm(ctx, mk(o, o, v, Iov, v, false, t1, v, true, Foo, o, 1.0, 1.0)));
      MISC(k_copy2d(1, v, v, Ivv, v, 0, Fvv, v, 0, false, s));
      RCHK(gemm(ctx, mk(v, v, o, t1, v, true, Iov, v, false, Fvv, v, -1.0, 1.0)));
      // Fvo = Ivo - t1^T Ioo + Fvv_part t1^T with Fvv_part = Ivv - t1^T Iov (= Fvv)
      MISC(k_copy2d(1, v, o, Ivo, o, 0, Fvo, o, 0, false, s));
      RCHK(gemm(ctx, mk(v, o, o, t1, v, true, Ioo, o, false, Fvo, o, -1.0, 1.0)));
      RCHK(gemm(ctx, mk(v, o, v, Fvv, v, false, t1, v, true, Fvo, o, 1.0, 1.0)));
    } else {
      MISC(k_copy2d(1, 1, n * n, ctx->Fin, n * n, 0, ctx->Fh, n * n, 0, false, s));
    }
  }

  // ---------------- assembly of the symmetric terms (Alg. 2, 3, 9) ----------------------------
  ctx->section = "gemm@assembly";
  ctx->chain = 1;
  ctx->mixed = ctx->want_mixed;
  RCHK(gemm(ctx, mk(P, P, P, ctx->S, P, false, T, P, false, ctx->ST, P)));
  if (mask & THC_TERM_EQ28) MISC(k_batch_sum_sym(ctx->KS, P, ctx->sig28, 1.0, ctx->sig, s));
  if (mask & THC_TERM_EQ29) {
    // sigma += Abar K^T + K Abar^T, K = Abar/2 + 2 S T Atil - H
    RCHK(gemm(ctx, mk(P, nL, P, ctx->ST, P, false, ctx->At, nL, false, ctx->K29, nL, 2.0, 0.0)));
    MISC(k_axpby(P * nL, 0.5, ctx->Abar, 1.0, ctx->K29, s));
    MISC(k_axpby(P * nL, -1.0, ctx->Hh, 1.0, ctx->K29, s));
    RCHK(gemm(ctx, mk(P, P, nL, ctx->Abar, nL, false, ctx->K29, nL, true, ctx->Qm, P)));
    MISC(k_sym_add(P, ctx->Qm, 1.0, ctx->sig, s));
  }
  if (mask & THC_TERM_EQ31) {
    // sigma -= S T C3^T + C3 T S
    RCHK(gemm(ctx, mk(P, P, P, ctx->ST, P, false, ctx->C3, P, true, ctx->Qm, P)));
    MISC(k_sym_add(P, ctx->Qm, -1.0, ctx->sig, s));
  }
  if (mask & THC_TERM_EQ41) {
    // Alg. 9: E = Go o vt - Gv o ot, vt = Yv^T (F^vv + xi_vv) Yv, ot = Yo^T (F^oo + xi_oo)^T Yo
    MISC(k_copy2d(1, o, o, Foo, o, 0, ctx->Fxoo, o, 0, false, s));
    MISC(k_axpby(o * o, 1.0, ctx->xioo, 1.0, ctx->Fxoo, s));
    MISC(k_copy2d(1, v, v, Fvv, v, 0, ctx->Fxvv, v, 0, false, s));
    MISC(k_axpby(v * v, 1.0, ctx->xivv, 1.0, ctx->Fxvv, s));
    RCHK(gemm(ctx, mk(o, P, o, ctx->Fxoo, o, true, Yo, P, false, ctx->tmpoP, P)));
    RCHK(gemm(ctx, mk(P, P, o, Yo, P, true, ctx->tmpoP, P, false, ctx->ot, P)));
    RCHK(gemm(ctx, mk(v, P, v, ctx->Fxvv, v, false, Yv, P, false, ctx->tmpvP, P)));
    RCHK(gemm(ctx, mk(P, P, v, Yv, P, true, ctx->tmpvP, P, false, ctx->vt, P)));
    MISC(k_hadamard(PP, ctx->Go, ctx->vt, 1.0, 0.0, ctx->E9, s));
    MISC(k_hadamard(PP, ctx->Gv, ctx->ot, -1.0, 1.0, ctx->E9, s));
    RCHK(gemm(ctx, mk(P, P, P, ctx->ST, P, false, ctx->E9, P, true, ctx->Qm, P)));
    MISC(k_sym_add(P, ctx->Qm, 1.0, ctx->sig, s));
  }

  // ---------------- Alg. 4 + 5: the same terms in O(N^5), all matrix products ---------------
  if ((mask & THC_TERM_EQ32) && ctx->quintic) {
    ctx->section = "gemm@alg45";
    ctx->chain = 2;
    RCHK(quintic_terms(ctx, T));
  }
  // ---------------- Alg. 6: quartic T2^2 ladder + exchange (Eq. 32 + 33) ----------------------
  ctx->section = "gemm@alg6";
  ctx->chain = 3;
  if ((mask & THC_TERM_EQ32) && !ctx->quintic) {
    const int64_t Xb = ctx->Xb, nX = Xb / 64;
    for (int64_t X0 = 0; X0 < P; X0 += Xb) {
      const int64_t xb = std::min(Xb, P - X0);
      // C6[i][Y][x] = sum_W T[W][Y] y_i^W Gv[X][W];  D6[a][Y][x] = sum_W T[W][Y] y_a^W Go[X][W]
      // stored [x/64][Y/2][x%64][Y%2] (X tiles of 64, row pairs interleaved: the H-kernel's layout)
      {
        Gemm g = batched(mk(P, xb, P, T, P, true, ctx->Gv + X0 * P, P, true, ctx->C6, Pp / 2), o, 0, 0, Xb * Pp);
        g.kscaleA = Yo; g.ksA = 1; g.sksA = P; g.pair_rows = true; g.xtile = true;
        RCHK(gemm(ctx, g));
        Gemm h = batched(mk(P, xb, P, T, P, true, ctx->Go + X0 * P, P, true, ctx->D6, Pp / 2), v, 0, 0, Xb * Pp);
        h.kscaleA = Yv; h.ksA = 1; h.sksA = P; h.pair_rows = true; h.xtile = true;
        RCHK(gemm(ctx, h));
      }
      for (int64_t I0 = 0; I0 < Q; I0 += ctx->Ic) {
        const int64_t ic = std::min(ctx->Ic, Q - I0);
        // E_I = sum_i x_i^I C6[i];  F_I = sum_a x_a^I D6[a], one product per X tile, stored
        // [x/64][I][Y/2][x%64][Y%2] (a tile's rows for consecutive I are adjacent)
        {
          const int64_t tb = Pp * 64;  // elements of one X tile of C6[i], D6[a], E_I, F_I
          Gemm ge = batched(mk(ic, tb, o, xo + I0, Q, true, ctx->C6, Xb * Pp, false, ctx->Ec, tb), nX, 0, tb, ctx->Ic * tb);
          Gemm gf = batched(mk(ic, tb, v, xv + I0, Q, true, ctx->D6, Xb * Pp, false, ctx->Fc, tb), nX, 0, tb, ctx->Ic * tb);
          if (ctx->mixed) {  // FP32 operands for the H-kernel
            ge.C = nullptr; ge.Cf = ctx->Ec32;
            gf.C = nullptr; gf.Cf = ctx->Fc32;
          }
          RCHK(gemm(ctx, ge));
          RCHK(gemm(ctx, gf));
        }
        // G_I[Y][Z] = sum_ia y_i^Y y_a^Z B_ia^I   (Alg. 6), stored in 16 x H_GBLK blocks (FP64) or
        // in 16 x 16 blocks (FP32, mixed precision)
        RCHK(gemm(ctx, mk(ic * o, P, v, ctx->Bq + I0 * ov, v, false, Yv, P, false, ctx->GYc, P)));
        if (ctx->mixed) {
          Gemm gg = batched(mk(P, P, o, Yo, P, true, ctx->GYc, P, false, nullptr, Pp), ic, 0, o * P, Pp * Pp);
          gg.Cf = ctx->G32;
          gg.cblk = 16;
          RCHK(gemm(ctx, gg));
        } else {
          Gemm gg = batched(mk(P, P, o, Yo, P, true, ctx->GYc, P, false, ctx->Gc, Pp), ic, 0, o * P, Pp * Pp);
          gg.cblk = H_GBLK;
          RCHK(gemm(ctx, gg));
        }
        if (ctx->mixed) {
          Scope sc(ctx, "h_kernel");
          sc.launches = ctx->nhtiles32 / (8 * ctx->hslots32);
          HIPCHK(h_accumulate_f32(Pp, Xb, ctx->Ic, ic, ctx->Ec32, ctx->Fc32, ctx->G32, ctx->Hb, ctx->htiles32,
                                  ctx->nhtiles32, ctx->hslots32, I0 == 0, s));
        } else {
          Scope sc(ctx, "h_kernel");
          sc.launches = ctx->nhtiles / (8 * ctx->hslots);  // one dispatch per generation of tiles
          HIPCHK(h_accumulate(Pp, Xb, ctx->Ic, ic, ctx->Ec, ctx->Fc, ctx->Gc, ctx->Hb, ctx->htiles, ctx->nhtiles,
                              ctx->hslots, I0 == 0, s));
        }
      }
      // I^X_ia = sum_YZ y_i^Z y_a^Y H^XYZ ; sigma^XW += sum_ia y_i^W y_a^W I^X_ia  (Alg. 6)
      // with H stored [Y][Z][x]: R1[Y][i][x] = sum_Z y_i^Z H[Y][Z][x], I6[i][a][x] = sum_Y y_a^Y R1[Y][i][x]
      RCHK(gemm(ctx, batched(mk(o, xb, P, Yo, P, false, ctx->Hb, Xb, false, ctx->R1, Xb), P, 0, Pp * Xb, o * Xb)));
      RCHK(gemm(ctx, batched(mk(v, xb, P, Yv, P, false, ctx->R1, o * Xb, false, ctx->I6, Xb), o, 0, Xb, v * Xb)));
      RCHK(gemm(ctx, mk(xb, P, ov, ctx->I6, Xb, true, ctx->Bkr, P, false, ctx->sig + X0 * P, P, 1.0, 1.0)));
      RCHK(progress(ctx, "Alg. 6 H blocks", X0 / Xb + 1, (P + Xb - 1) / Xb));
    }
  }

  // ---------------- Alg. 7: T2^2 rings (Eq. 35-37) ------------------------------------------
  // Rows X of the P x o x Q intermediates are taken in chunks of X7 (the paper's split of Alg. 7
  // over X); S^X and R^X are held for every X (the products with them need every row).
  ctx->section = "gemm@alg7";
  ctx->chain = 4;
  if (mask & THC_TERM_EQ35) {
    const int64_t X7 = ctx->X7;
    // S^X_ia = - sum_YZ y_i^Y y_a^Z Gv[X][Y] Go[X][Z] T[Y][Z]  (Alg. 7)
    for (int64_t X0 = 0; X0 < P; X0 += X7) {
      const int64_t xc = std::min(X7, P - X0);
      Gemm g = batched(mk(o, P, P, Yo, P, false, T, P, false, ctx->U7, P), xc, 0, 0, o * P);
      g.kscaleA = ctx->Gv + X0 * P; g.ksA = 1; g.sksA = P;
      RCHK(gemm(ctx, g));
      Gemm h = batched(mk(o, v, P, ctx->U7, P, false, Yv, P, true, ctx->S7 + X0 * ov, v, -1.0, 0.0), xc, o * P, 0, ov);
      h.kscaleB = ctx->Go + X0 * P; h.ksB = 1; h.sksB = P;
      RCHK(gemm(ctx, h));
    }
    // R^X = 2 sum_Y y_i^Y y_a^Y (S T)[X][Y] + S^X  (Alg. 7, Eq. 36)
    MISC(k_copy2d(1, 1, P * ov, ctx->S7, P * ov, 0, ctx->R7, P * ov, 0, false, s));
    RCHK(gemm(ctx, mk(P, ov, P, ctx->ST, P, false, ctx->Bkr, P, true, ctx->R7, ov, 2.0, 1.0)));
    const bool fused = exch_supported(o) && !(ctx->opt.flags & THC_FLAG_UNFUSED_EXCHANGE);
    for (int64_t X0 = 0; X0 < P; X0 += X7) {
      const int64_t xc = std::min(X7, P - X0);
      // half-transformed: Rx[X][i][J] = sum_a R[X][i][a] x_a^J (and Sx)
      RCHK(gemm(ctx, mk(xc * o, Q, v, ctx->R7 + X0 * ov, v, false, xv, Q, false, ctx->Rx, Q)));
      RCHK(gemm(ctx, mk(xc * o, Q, v, ctx->S7 + X0 * ov, v, false, xv, Q, false, ctx->Sx, Q)));
      // C^XI = sum_ia x_i^I x_a^I R^X_ia  (Alg. 7, Eq. 37)
      MISC(k_diag_eri(xc, Q, o, xo, ctx->Rx, ctx->Cx + X0 * Q, s));
      // exchange parts (Alg. 7): fused on chip when o fits the kernel's tile, else two GEMMs per X
      if (fused) {
        Scope sc(ctx, "exch");
        HIPCHK(exch_fused(o, Q, xc, xo, ctx->z, ctx->Rx, ctx->Gt, ctx->mixed, s));
        HIPCHK(exch_fused(o, Q, xc, xo, ctx->z, ctx->Sx, ctx->Gts, ctx->mixed, s));
      } else {
        for (int64_t x0 = 0; x0 < xc; x0 += ctx->Xc) {
          const int64_t xn = std::min(ctx->Xc, xc - x0);
          for (int pass = 0; pass < 2; ++pass) {
            const double* src = pass == 0 ? ctx->Rx : ctx->Sx;
            double* dst = pass == 0 ? ctx->Gt : ctx->Gts;
            // F^IJ = z^IJ sum_i x_i^I Rx[X][i][J]
            Gemm g = batched(mk(Q, Q, o, xo, Q, true, src + x0 * o * Q, Q, false, ctx->F7, Q), xn, 0, o * Q, Q * Q);
            g.hmul = ctx->z; g.ldh = Q; g.sH = 0;
            RCHK(gemm(ctx, g));
            // Gt[X][i][I] = sum_J x_i^J F^IJ
            RCHK(gemm(ctx, batched(mk(o, Q, Q, xo, Q, false, ctx->F7, Q, true, dst + x0 * o * Q, Q), xn, 0, Q * Q, o * Q)));
          }
        }
      }
      // G^X_ia = sum_I Gt[X][i][I] x_a^I ; sigma[X] += c_D ( - G R^T + G~ S^T )
      RCHK(gemm(ctx, mk(xc * o, v, Q, ctx->Gt, Q, false, xv, Q, true, ctx->G7, v)));
      RCHK(gemm(ctx, mk(xc * o, v, Q, ctx->Gts, Q, false, xv, Q, true, ctx->G7s, v)));
      RCHK(gemm(ctx, mk(xc, P, ov, ctx->G7, ov, false, ctx->R7, ov, true, ctx->sig + X0 * P, P, -C_D, 1.0)));
      RCHK(gemm(ctx, mk(xc, P, ov, ctx->G7s, ov, false, ctx->S7, ov, true, ctx->sig + X0 * P, P, C_D, 1.0)));
      RCHK(progress(ctx, "Alg. 7 row chunks", X0 / X7 + 1, (P + X7 - 1) / X7));
    }
    // D = C z ; sigma += 2 c_D C D^T  (Alg. 7, Eq. 37)
    RCHK(gemm(ctx, mk(P, Q, Q, ctx->Cx, Q, false, ctx->z, Q, false, ctx->Dx, Q)));
    RCHK(gemm(ctx, mk(P, P, Q, ctx->Cx, Q, false, ctx->Dx, Q, true, ctx->sig, P, 2.0 * C_D, 1.0)));
  }

  // ---------------- singles residual (Alg. 8, Alg. 10) ---------------------------------------
  ctx->section = "gemm@singles";
  ctx->chain = 5;
  if (sres && (mask & THC_TERM_EQ38)) {
    // s38 was accumulated with undressed Lvv/Loo; the dressing adds -xi_oo^T t1 + t1 xi_vv^T
    MISC(k_axpby(ov, 1.0, ctx->s38, 1.0, ctx->sig1, s));
    if (singles) {
      RCHK(gemm(ctx, mk(o, v, o, ctx->xioo, o, true, t1, v, false, ctx->sig1, v, -1.0, 1.0)));
      RCHK(gemm(ctx, mk(o, v, v, t1, v, false, ctx->xivv, v, true, ctx->sig1, v, 1.0, 1.0)));
    }
  }
  if (singles) {  // with t1 = 0 the Fock matrix is diag(eps) and these terms vanish
    if (mask & THC_TERM_EQ42) {
      // F^_ai + 2 Yo diag(T f) Yv^T - Yo (T o Mf^T) Yv^T, Mf = Yo^T F^ov Yv, f = diag(Mf)
      MISC(k_copy2d(1, o, v, Fvo, o, 0, ctx->tmpov, v, 0, true, s));
      MISC(k_axpby(ov, 1.0, ctx->tmpov, 1.0, ctx->sig1, s));
      RCHK(gemm(ctx, mk(o, P, v, Fov, v, false, Yv, P, false, ctx->tmpoP, P)));
      RCHK(gemm(ctx, mk(P, P, o, ctx->tmpoP, P, true, Yo, P, false, ctx->Qm, P)));  // Mf^T
      MISC(k_diag(P, ctx->Qm, P, ctx->fd, s));
      MISC(k_gemv(P, P, T, P, ctx->fd, ctx->Tf, s));
      MISC(k_hadamard(PP, T, ctx->Qm, 1.0, 0.0, ctx->E9, s));
      RCHK(gemm(ctx, mk(o, P, P, Yo, P, false, ctx->E9, P, false, ctx->tmpoP, P)));
      RCHK(gemm(ctx, mk(o, v, P, ctx->tmpoP, P, false, Yv, P, true, ctx->sig1, v, -1.0, 1.0)));
      Gemm g = mk(o, v, P, Yo, P, false, Yv, P, true, ctx->sig1, v, 2.0, 1.0);
      g.kscaleA = ctx->Tf; g.ksA = 1;
      RCHK(gemm(ctx, g));
    }
  }
  ctx->section = nullptr;
  ctx->chain = -1;
  return THC_OK;
}

double energy_from_scalars(const double* h, bool singles) {
  // E = 2 Atil^T T Atil - sum T o M o M^T  (+ singles: 2 sum d_A^2 - sum tr K_A^2)
  double e = 2.0 * h[0] - h[1];
  if (singles) e += 2.0 * h[2] - h[3];
  return e;
}

// sigma^ = W^T sigma W (into ctx->sigh) and the norms of sigma^ and sigma1 into scal[8], scal[9].
int project_basis(thc_ctx* ctx) {
  const int64_t P = ctx->P;
  RCHK(gemm(ctx, mk(P, P, P, ctx->sig, P, false, ctx->W, P, false, ctx->Qm, P)));
  RCHK(gemm(ctx, mk(P, P, P, ctx->W, P, true, ctx->Qm, P, false, ctx->sigh, P)));
  MISC(k_dot(P * P, ctx->sigh, ctx->sigh, ctx->scal + 8, ctx->stream));
  MISC(k_dot(ctx->ov, ctx->sig1, ctx->sig1, ctx->scal + 9, ctx->stream));
  return THC_OK;
}

// Z = W T^ W^T
int raw_from_basis(thc_ctx* ctx, const double* Th, double* Z) {
  const int64_t P = ctx->P;
  RCHK(gemm(ctx, mk(P, P, P, Th, P, false, ctx->W, P, true, ctx->Qm, P)));
  RCHK(gemm(ctx, mk(P, P, P, ctx->W, P, false, ctx->Qm, P, false, Z, P)));
  return THC_OK;
}

// T^ = W^T S Z S W
int basis_from_raw(thc_ctx* ctx, const double* Z, double* Th) {
  const int64_t P = ctx->P;
  RCHK(gemm(ctx, mk(P, P, P, ctx->S, P, false, ctx->W, P, false, ctx->Qm, P)));    // S W
  RCHK(gemm(ctx, mk(P, P, P, Z, P, false, ctx->Qm, P, false, ctx->E9, P)));         // Z S W
  RCHK(gemm(ctx, mk(P, P, P, ctx->Qm, P, true, ctx->E9, P, false, Th, P)));         // W^T S Z S W
  return THC_OK;
}

int need_built(thc_ctx* ctx) {
  if (!ctx->built) {
    ctx->err = "thc_build_factors has not completed";
    return THC_ESTATE;
  }
  return THC_OK;
}

}  // namespace

// =========================================================================================
namespace {
// Solves (A + ridge max|diag A| I) x = b for a symmetric positive semi-definite A (overwritten).
bool spd_solve(int64_t n, std::vector<double>& A, std::vector<double>& b, double ridge) {
  double dmax = 0.0;
  for (int64_t i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(A[(size_t)i * n + i]));
  if (!(dmax > 0.0)) dmax = 1.0;
  for (int64_t i = 0; i < n; ++i) A[(size_t)i * n + i] += ridge * dmax;
  if (host_cholesky(n, A.data()) != 0) return false;
  for (int64_t i = 0; i < n; ++i) {  // L y = b
    double acc = b[i];
    for (int64_t k = 0; k < i; ++k) acc -= A[(size_t)i * n + k] * b[k];
    b[i] = acc / A[(size_t)i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {  // L^T x = y
    double acc = b[i];
    for (int64_t k = i + 1; k < n; ++k) acc -= A[(size_t)k * n + i] * b[k];
    b[i] = acc / A[(size_t)i * n + i];
  }
  return true;
}
}  // namespace

struct thc_mlp {
  int64_t n_in = 0, w = 0, n_out = 0, np = 0;
  void* pin = nullptr;  // pinned host staging buffer
  size_t pin_bytes = 0;
  hipStream_t stream = nullptr;
  std::string err;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  float *mu_in = nullptr, *sd_in = nullptr, *mu_out = nullptr, *sd_out = nullptr, *loss = nullptr;
  double* part = nullptr;
  int64_t step = 0;
  // activations for up to `cap` rows
  int64_t cap = 0;
  float *xn = nullptr, *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *yn = nullptr, *dy = nullptr,
        *d2 = nullptr, *d1 = nullptr;
  short* wb = nullptr;
  float* bb = nullptr;
  bool packed = false;
  float* scratch = nullptr;            // device address of the allocation-free pass's scratch
  hipError_t scratch_err = hipSuccess;  // why it could not be looked up, if it could not
  std::vector<void*> allocs, acts;
};

namespace {
constexpr int64_t MLP_PARTS = 1024;

template <class T>
int mlp_alloc(thc_mlp* ctx, T** p, size_t count, std::vector<void*>& list) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "hipMalloc failed";
    return THC_ENOMEM;
  }
  list.push_back(q);
  *p = (T*)q;
  return THC_OK;
}

int mlp_reserve(thc_mlp* ctx, int64_t rows) {
  if (rows <= ctx->cap) return THC_OK;
  for (void* q : ctx->acts) (void)hipFree(q);
  ctx->acts.clear();
  const int64_t R = std::max<int64_t>(rows, 1024), w = ctx->w;
  RCHK(mlp_alloc(ctx, &ctx->xn, (size_t)(R * ctx->n_in), ctx->acts));
  for (float** a : {&ctx->z1, &ctx->h1, &ctx->z2, &ctx->h2, &ctx->d2, &ctx->d1})
    RCHK(mlp_alloc(ctx, a, (size_t)(R * w), ctx->acts));
  RCHK(mlp_alloc(ctx, &ctx->yn, (size_t)(R * ctx->n_out), ctx->acts));
  RCHK(mlp_alloc(ctx, &ctx->dy, (size_t)(R * ctx->n_out), ctx->acts));
  ctx->cap = R;
  return THC_OK;
}

// Activations of one FP32 forward pass of R rows.
struct MlpActs {
  float *xn, *z1, *h1, *z2, *h2, *yn;
};

// forward in FP32 into a: xn, z1, h1, z2, h2, yn (normalized outputs)
int mlp_fwd_into(thc_mlp* ctx, const float* X, int64_t R, const MlpActs& a) {
  const int64_t ni = ctx->n_in, w = ctx->w, no = ctx->n_out;
  const float *W1 = ctx->p, *b1 = W1 + ni * w, *W2 = b1 + w, *b2 = W2 + w * w, *W3 = b2 + w, *b3 = W3 + w * no;
  hipStream_t s = ctx->stream;
  HIPCHK(mlp_normalize(R, ni, X, ctx->mu_in, ctx->sd_in, a.xn, s));
  HIPCHK(mlp_sgemm(false, false, 1, R, w, ni, a.xn, ni, W1, w, a.h1, w, b1, a.z1, w, s));
  HIPCHK(mlp_sgemm(false, false, 1, R, w, w, a.h1, w, W2, w, a.h2, w, b2, a.z2, w, s));
  HIPCHK(mlp_sgemm(false, false, 2, R, no, w, a.h2, w, W3, no, a.yn, no, b3, nullptr, 0, s));
  return THC_OK;
}

// Rows of one allocation-free forward pass that fit the scratch array: xn, h1, h2 and yn, each
// starting on a 64-float (256-byte) boundary.
int64_t mlp_scratch_floats(const thc_mlp* ctx, int64_t R) {
  auto up = [](int64_t n) { return (n + 63) / 64 * 64; };
  return up(R * ctx->n_in) + 2 * up(R * ctx->w) + up(R * ctx->n_out);
}

int64_t mlp_scratch_rows(const thc_mlp* ctx) {
  const int64_t per = ctx->n_in + 2 * ctx->w + ctx->n_out;
  int64_t r = MLP_SCRATCH_FLOATS / per;
  while (r > 0 && mlp_scratch_floats(ctx, r) > MLP_SCRATCH_FLOATS) --r;
  return r;
}

// forward in FP32 into the network's own activation buffers
int mlp_fwd(thc_mlp* ctx, const float* X, int64_t R) {
  return mlp_fwd_into(ctx, X, R, MlpActs{ctx->xn, ctx->z1, ctx->h1, ctx->z2, ctx->h2, ctx->yn});
}

// loss and gradient (into ctx->g) of the mean squared error on normalized targets
int mlp_bwd(thc_mlp* ctx, const float* X, const float* T, int64_t R) {
  const int64_t ni = ctx->n_in, w = ctx->w, no = ctx->n_out;
  const float *W2 = ctx->p + ni * w + w, *W3 = W2 + w * w + w;
  float *gW1 = ctx->g, *gb1 = gW1 + ni * w, *gW2 = gb1 + w, *gb2 = gW2 + w * w, *gW3 = gb2 + w, *gb3 = gW3 + w * no;
  hipStream_t s = ctx->stream;
  RCHK(mlp_fwd(ctx, X, R));
  HIPCHK(mlp_mse_grad(R, no, ctx->yn, T, ctx->mu_out, ctx->sd_out, ctx->dy, ctx->part, MLP_PARTS, ctx->loss, s));
  HIPCHK(mlp_sgemm(true, false, 0, w, no, R, ctx->h2, w, ctx->dy, no, gW3, no, nullptr, nullptr, 0, s));
  HIPCHK(mlp_colsum(R, no, ctx->dy, gb3, s));
  HIPCHK(mlp_sgemm(false, true, 3, R, w, no, ctx->dy, no, W3, no, ctx->d2, w, nullptr, ctx->z2, w, s));
  HIPCHK(mlp_sgemm(true, false, 0, w, w, R, ctx->h1, w, ctx->d2, w, gW2, w, nullptr, nullptr, 0, s));
  HIPCHK(mlp_colsum(R, w, ctx->d2, gb2, s));
  HIPCHK(mlp_sgemm(false, true, 3, R, w, w, ctx->d2, w, W2, w, ctx->d1, w, nullptr, ctx->z1, w, s));
  HIPCHK(mlp_sgemm(true, false, 0, ni, w, R, ctx->xn, ni, ctx->d1, w, gW1, w, nullptr, nullptr, 0, s));
  HIPCHK(mlp_colsum(R, w, ctx->d1, gb1, s));
  return THC_OK;
}

}  // namespace

extern "C" {

namespace {
bool options_valid(const thc_options* opt) {
  if (opt->o < 1 || opt->v < 1 || opt->nL < 1 || opt->nP < 1 || opt->nQ < 1 || opt->diis_max < 0 ||
      opt->diis_max > 16 || (opt->precision < 0 || opt->precision > 2) ||
      (opt->flags & ~(THC_FLAG_UNFUSED_EXCHANGE | THC_FLAG_STREAM_LVV | THC_FLAG_PROGRESS | THC_FLAG_QUINTIC |
                      THC_FLAG_QUARTIC | THC_FLAG_CHECK)) != 0 || ((opt->flags & THC_FLAG_QUINTIC) && (opt->flags & THC_FLAG_QUARTIC)) || opt->a_block < 0 ||
      opt->i_chunk < 0 || opt->x_block < 0 || opt->x_chunk < 0 || opt->x7_chunk < 0 || opt->q_pairs < 0 ||
      opt->q_jchunk < 0 || (opt->split_mask & ~(uint64_t)THC_CHAIN_ALL) != 0 || opt->guess < 0 || opt->guess > 1)
    return false;
  // the metric S = B^T B (nP x nP) and the ERI-grid Gram (nQ x nQ) have rank at most o v
  return opt->nP <= opt->o * opt->v && opt->nQ <= opt->o * opt->v;
}

void fill_plan_info(const thc_ctx* ctx, int64_t tiles, int64_t entries, int64_t slots, double bytes, thc_plan_info* out) {
  thc_plan_info p{};
  p.a_block = ctx->nb;
  p.alg1_splits = ctx->KS;
  p.alg1_tile = ctx->alg1_tile;
  p.x_block = ctx->Xb;
  p.x_blocks = (ctx->P + ctx->Xb - 1) / ctx->Xb;
  p.i_chunk = ctx->Ic;
  p.i_chunks = (ctx->Q + ctx->Ic - 1) / ctx->Ic;
  p.h_generations = entries / (8 * slots);
  p.h_tiles = tiles;
  p.x_chunk = ctx->Xc;
  p.x7_chunk = ctx->X7;
  p.x7_chunks = (ctx->P + ctx->X7 - 1) / ctx->X7;
  p.exchange_fused = exch_supported(ctx->o) && !(ctx->opt.flags & THC_FLAG_UNFUSED_EXCHANGE);
  p.lvv_resident = ctx->lvv_resident ? 1 : 0;
  p.quintic = ctx->quintic ? 1 : 0;
  p.q_pairs = ctx->quintic ? ctx->nq : 0;
  p.q_jchunk = ctx->quintic ? ctx->jq : 0;
  p.device_bytes = (uint64_t)bytes;
  *out = p;
}
}  // namespace

int thc_create_with_workspace(const thc_options* opt, void* dev_workspace, size_t ws_bytes, void* stream,
                              thc_ctx** out) {
  if (!opt || !out || !dev_workspace || ws_bytes == 0 || ((uintptr_t)dev_workspace % 256) != 0) return THC_EINVAL;
  const int rc = thc_create(opt, stream, out);
  if (rc != THC_OK) return rc;
  (*out)->ws = dev_workspace;
  (*out)->ws_bytes = ws_bytes;
  return THC_OK;
}

int thc_plan_query(const thc_options* opt, int synthetic, uint64_t budget_bytes, thc_plan_info* out) {
  if (!opt || !out || !options_valid(opt) || budget_bytes == 0) return THC_EINVAL;
  thc_ctx c;
  c.opt = *opt;
  c.o = opt->o; c.v = opt->v; c.n = opt->o + opt->v; c.nL = opt->nL;
  c.P = opt->nP; c.Q = opt->nQ; c.ov = opt->o * opt->v;
  c.synth = synthetic != 0;
  int64_t slots = h_slots_per_xcd();  // from the current device when there is one
  if (slots < 1) {
    (void)hipGetLastError();
    slots = 64;  // 32 CUs per XCD, two H-kernel workgroups per CU (MI355X)
  }
  const int rc = choose_plan(&c, (double)budget_bytes, slots);
  if (rc != THC_OK) return rc;
  const double pers = list_bytes(persistent_list(&c)),
               r6 = list_bytes(c.quintic ? quintic_list(&c) : region6_list(&c));
  const double a7 = list_bytes(alg7_list(&c)), setup = 8.0 * (double)setup_doubles(&c);
  int64_t tiles = 0, entries = 0;
  tile_counts(c.Pp, c.Xb, slots, &tiles, &entries);
  fill_plan_info(&c, tiles, entries, slots,
                 pers + 8.0 * (double)tile_table_doubles(c.Pp, c.Xb, slots) * (opt->precision >= 1 ? 2.0 : 1.0) +
                     std::max(r6, setup) + a7,
                 out);
  return THC_OK;
}

int thc_create(const thc_options* opt, void* stream, thc_ctx** out) {
  if (!opt || !out) return THC_EINVAL;
  *out = nullptr;
  if (!options_valid(opt)) return THC_EINVAL;
  thc_ctx* ctx = new (std::nothrow) thc_ctx();
  if (!ctx) return THC_ENOMEM;
  ctx->opt = *opt;
  ctx->stream = (hipStream_t)stream;
  ctx->o = opt->o; ctx->v = opt->v; ctx->n = opt->o + opt->v; ctx->nL = opt->nL;
  ctx->P = opt->nP; ctx->Q = opt->nQ; ctx->ov = opt->o * opt->v;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return THC_EDEVICE;
  }
  *out = ctx;
  return THC_OK;
}

namespace {
// Synthetic inputs generated into the library layout (the twin of the Python generator): orbital
// energies on the host, factors and Cholesky blocks on the device, and the global scale gamma
// (given, or from lambda_max(L_ov L_ov^T) by power iteration on the nL x nL Gram matrix).
int generate_inputs(thc_ctx* ctx) {
  hipStream_t s = ctx->stream;
  const int64_t o = ctx->o, v = ctx->v, n = ctx->n, nL = ctx->nL, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const thc_synth_spec& sp = ctx->spec;
  std::vector<double> e(n);
  synth_energies(sp.seed, o, v, e.data());
  RCHK(h2d(ctx, ctx->eps, e.data(), n * sizeof(double)));
  const double sP = std::sqrt((double)P), sQ = std::sqrt((double)Q);
  MISC(synth_normals(sp.seed, thc_synth_stream_xo_amp, 0, o * P, sP, ctx->Yo, s));
  MISC(synth_normals(sp.seed, thc_synth_stream_xv_amp, 0, v * P, sP, ctx->Yv, s));
  MISC(synth_normals(sp.seed, thc_synth_stream_xo_eri, 0, o * Q, sQ, ctx->xo, s));
  MISC(synth_normals(sp.seed, thc_synth_stream_xv_eri, 0, v * Q, sQ, ctx->xv, s));
  // unscaled oo and ov blocks, then gamma
  MISC(synth_chol_block(sp.seed, n, 0, nL, 0, o, 0, o, sp.decay, 1.0, ctx->Loo, s));
  MISC(synth_chol_block(sp.seed, n, 0, nL, 0, o, o, v, sp.decay, 1.0, ctx->Lov, s));
  double gamma = sp.gamma;
  if (!(gamma > 0.0)) {
    // the rule's Gram matrix and vectors at the start of the set-up scratch
    double* G = ctx->setup_scratch;
    double* x = G + aligned((size_t)(nL * nL));
    double* y = x + aligned((size_t)nL);
    auto tfree = [&]() {};
    int rc = gemm(ctx, mk(nL, nL, ov, ctx->Lov, ov, false, ctx->Lov, ov, true, G, nL));
    if (rc == THC_OK) {
      std::vector<double> ones((size_t)nL, 1.0 / std::sqrt((double)nL));
      rc = h2d(ctx, x, ones.data(), nL * sizeof(double));
    }
    for (int it = 0; it < 200 && rc == THC_OK; ++it) {
      if (k_gemv(nL, nL, G, nL, x, y, s) != hipSuccess || k_dot(nL, y, y, ctx->scal + 60, s) != hipSuccess ||
          synth_normalize(nL, y, ctx->scal + 60, x, s) != hipSuccess) {
        ctx->err = "gamma rule: kernel launch failed";
        rc = THC_EDEVICE;
      }
    }
    double lam2 = 0.0;
    if (rc == THC_OK) rc = d2h(ctx, &lam2, ctx->scal + 60, sizeof(double));
    tfree();
    RCHK(rc);
    const double lam = std::sqrt(lam2);
    const double dmin = 2.0 * (e[o] - e[o - 1]);
    if (!(lam > 0.0) || !(dmin > 0.0)) { ctx->err = "gamma rule: degenerate inputs"; return THC_ENUMERIC; }
    gamma = std::sqrt(sp.coupling * dmin / lam);
  }
  ctx->gamma = gamma;
  MISC(synth_scale(nL * o * o, gamma, ctx->Loo, s));
  MISC(synth_scale(nL * ov, gamma, ctx->Lov, s));
  if (ctx->lvv_resident) MISC(synth_chol_block(sp.seed, n, 0, nL, o, v, o, v, sp.decay, gamma, ctx->Lvv, s));
  return THC_OK;
}
}  // namespace

int thc_set_synthetic(thc_ctx* ctx, const thc_synth_spec* spec) {
  if (!ctx) return THC_EINVAL;
  if (!spec || !(spec->decay > 0.0) || (!(spec->gamma > 0.0) && !(spec->coupling > 0.0))) {
    ctx->err = "thc_set_synthetic: decay must be positive, and coupling too unless gamma is given";
    return THC_EINVAL;
  }
  if (ctx->built) { ctx->err = "factors already built for this context"; return THC_ESTATE; }
  ctx->synth = true;
  ctx->spec = *spec;
  return THC_OK;
}

int thc_synth_gamma(const thc_ctx* ctx, double* gamma) {
  if (!ctx || !gamma) return THC_EINVAL;
  if (!ctx->built) return THC_ESTATE;
  *gamma = ctx->synth ? ctx->gamma : 0.0;
  return THC_OK;
}

int thc_synth_normals(uint64_t seed, int32_t stream_id, uint64_t first, int64_t count, double divisor, double* out,
                      void* stream) {
  if (stream_id < 0 || stream_id > 6 || count < 0 || (count > 0 && !out) || divisor == 0.0) return THC_EINVAL;
  return synth_normals(seed, (uint64_t)stream_id, first, count, divisor, out, (hipStream_t)stream) == hipSuccess
             ? THC_OK
             : THC_EDEVICE;
}

int thc_synth_cholesky(uint64_t seed, int64_t n, int64_t K0, int64_t nK, double decay, double gamma, double* L,
                       void* stream) {
  if (n < 1 || K0 < 0 || nK < 0 || !(decay > 0.0) || (nK > 0 && !L)) return THC_EINVAL;
  return synth_chol_block(seed, n, K0, nK, 0, n, 0, n, decay, gamma, L, (hipStream_t)stream) == hipSuccess
             ? THC_OK
             : THC_EDEVICE;
}

int thc_synth_energies(uint64_t seed, int64_t o, int64_t v, double* eps) {
  if (o < 1 || v < 1 || !eps) return THC_EINVAL;
  synth_energies(seed, o, v, eps);
  return THC_OK;
}

int thc_build_factors(thc_ctx* ctx, const double* L, const double* eps, const double* X, double* Zout) {
  if (!ctx) return THC_EINVAL;
  if (!ctx->synth && (!L || !eps || !X)) { ctx->err = "null input"; return THC_EINVAL; }
  if (ctx->built) { ctx->err = "factors already built for this context"; return THC_ESTATE; }
  hipStream_t s = ctx->stream;
  RCHK(plan_and_alloc(ctx));
  const int64_t o = ctx->o, v = ctx->v, n = ctx->n, nL = ctx->nL, P = ctx->P, Q = ctx->Q, ov = ctx->ov;
  const int64_t PP = P * P;
  if (ctx->synth) {
    RCHK(generate_inputs(ctx));
  } else {
    // integrals and factors into the library layout
    MISC(k_copy2d(nL, o, o, L, n, n * n, ctx->Loo, o, o * o, false, s));
    MISC(k_copy2d(nL, o, v, L + o, n, n * n, ctx->Lov, v, ov, false, s));
    MISC(k_copy2d(nL, v, v, L + o * n + o, n, n * n, ctx->Lvv, v, v * v, false, s));
    HIPCHK(hipMemcpyAsync(ctx->eps, eps, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->Yo, X, o * P * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->Yv, X + o * P, v * P * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->xo, X + (o + v) * P, o * Q * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->xv, X + (o + v) * P + o * Q, v * Q * sizeof(double), hipMemcpyDeviceToDevice, s));
  }

  // Grams and metric (Eq. 10): S = (Xo^T Xo) o (Xv^T Xv); Khatri-Rao B[(ia)][X]
  RCHK(gemm(ctx, mk(P, P, o, ctx->Yo, P, true, ctx->Yo, P, false, ctx->Go, P)));
  RCHK(gemm(ctx, mk(P, P, v, ctx->Yv, P, true, ctx->Yv, P, false, ctx->Gv, P)));
  MISC(k_hadamard(PP, ctx->Go, ctx->Gv, 1.0, 0.0, ctx->S, s));
  MISC(k_kr(o, v, P, ctx->Yo, ctx->Yv, ctx->Bkr, s));

  // scratch for the set-up: pieces of the set-up region of the arena (sized by setup_doubles for
  // exactly the pieces taken below)
  size_t sused = ctx->synth ? aligned((size_t)(nL * nL)) + 2 * aligned((size_t)nL) : 0;  // the gamma rule's
  auto salloc = [&](size_t cnt) -> double* {
    if (sused + aligned(cnt) > ctx->setup_len) return nullptr;
    double* q = ctx->setup_scratch + sused;
    sused += aligned(cnt);
    return q;
  };
  auto sfree = [&]() {};
  int rc = THC_OK;
  do {
    // ---- ERI fit (Eq. 19-20): G_Q xi^T = M, M^IA = sum_ia x_i^I x_a^I L_ia^A, z = xi^T xi ----
    const int64_t CBn = (std::max(Q, P) + CB - 1) / CB;
    double* GQ = salloc(Q * Q);
    double* tmpQ = salloc(Q * Q);
    double* Linv = salloc(CBn * CB * CB);
    double* Mq = salloc(Q * nL);
    double* Tl = salloc(std::min<int64_t>(nL, 256) * o * Q);
    double* tmpw = salloc(std::max(Q, P) * std::max<int64_t>(std::max(nL, P), CB));
    double* tsolve = salloc(CB * std::max(std::max(nL, P), Q));  // panel / block-row scratch
    if (!GQ || !tmpQ || !Linv || !Mq || !Tl || !tmpw || !tsolve) { ctx->err = "set-up allocation failed"; rc = THC_ENOMEM; break; }
    rc = gemm(ctx, mk(Q, Q, o, ctx->xo, Q, true, ctx->xo, Q, false, GQ, Q)); if (rc) break;
    rc = gemm(ctx, mk(Q, Q, v, ctx->xv, Q, true, ctx->xv, Q, false, tmpQ, Q)); if (rc) break;
    MISC(k_hadamard(Q * Q, GQ, tmpQ, 1.0, 0.0, GQ, s));
    // M^T[A][I] in chunks of A: Tl[A][i][I] = sum_a L_ia^A x_a^I, then the diagonal contraction with xo
    for (int64_t A0 = 0; A0 < nL && rc == THC_OK; A0 += 256) {
      const int64_t na = std::min<int64_t>(256, nL - A0);
      rc = gemm(ctx, mk(na * o, Q, v, ctx->Lov + A0 * ov, v, false, ctx->xv, Q, false, Tl, Q));
      if (rc) break;
      MISC(k_diag_eri(na, Q, o, ctx->xo, Tl, tmpw + A0 * Q, s));  // tmpw holds M^T (nL x Q)
    }
    if (rc) break;
    MISC(k_copy2d(1, Q, nL, tmpw, Q, 0, Mq, nL, 0, true, s));  // M (Q x nL)
    rc = potrf(ctx, GQ, Q, Linv, tsolve, "the ERI grid metric G_Q"); if (rc) break;
    rc = trsm(ctx, GQ, Q, Linv, Mq, nL, false, tsolve); if (rc) break;
    rc = trsm(ctx, GQ, Q, Linv, Mq, nL, true, tsolve); if (rc) break;   // Mq = xi^T (Q x nL)
    rc = gemm(ctx, mk(Q, Q, nL, Mq, nL, false, Mq, nL, true, ctx->z, Q)); if (rc) break;
    // B_ia^I = sum_J x_i^J x_a^J z^IJ  (Alg. 6), layout [I][i][a]
    {
      Gemm g = batched(mk(Q, v, Q, ctx->z, Q, false, ctx->xv, Q, true, ctx->Bq, ov), o, 0, 0, v);
      g.kscaleB = ctx->xo; g.ksB = 1; g.sksB = Q;
      rc = gemm(ctx, g); if (rc) break;
    }

    rc = progress(ctx, "set-up: ERI fit and B_ia^I done, steps", 1, 3); if (rc) break;
    // ---- working basis: E_mat w = e S w, E_mat = Go o (Xv^T eps_v Xv) - (Xo^T eps_o Xo) o Gv ----
    double* Sl = salloc(PP);
    double* Em = salloc(PP);
    double* tP = salloc(PP);
    if (!Sl || !Em || !tP) { ctx->err = "set-up allocation failed"; rc = THC_ENOMEM; break; }
    {
      Gemm g = mk(P, P, v, ctx->Yv, P, true, ctx->Yv, P, false, Em, P);
      g.kscaleA = ctx->eps + o; g.ksA = 1;
      rc = gemm(ctx, g); if (rc) break;
      MISC(k_hadamard(PP, ctx->Go, Em, 1.0, 0.0, Em, s));
      Gemm h = mk(P, P, o, ctx->Yo, P, true, ctx->Yo, P, false, tP, P);
      h.kscaleA = ctx->eps; h.ksA = 1;
      rc = gemm(ctx, h); if (rc) break;
      MISC(k_hadamard(PP, tP, ctx->Gv, -1.0, 1.0, Em, s));
    }
    MISC(k_copy2d(1, P, P, ctx->S, P, 0, Sl, P, 0, false, s));
    rc = potrf(ctx, Sl, P, Linv, tsolve, "the amplitude metric S"); if (rc) break;
    // C = L^-1 E L^-T : Y = L^-1 E, C = L^-1 Y^T
    rc = trsm(ctx, Sl, P, Linv, Em, P, false, tsolve); if (rc) break;
    MISC(k_copy2d(1, P, P, Em, P, 0, tmpw, P, 0, true, s));
    rc = trsm(ctx, Sl, P, Linv, tmpw, P, false, tsolve); if (rc) break;
    std::vector<double> hC(PP), hw(P);
    rc = d2h(ctx, hC.data(), tmpw, PP * sizeof(double)); if (rc) break;
    for (int64_t i = 0; i < P; ++i)
      for (int64_t j = 0; j < i; ++j) {
        const double a = 0.5 * (hC[i * P + j] + hC[j * P + i]);
        hC[i * P + j] = a;
        hC[j * P + i] = a;
      }
    if (host_syev(P, hC.data(), hw.data()) != 0) { ctx->err = "eigensolver did not converge"; rc = THC_ENUMERIC; break; }
    if (hw[0] <= 0.0) { ctx->err = "projected Fock operator is not positive"; rc = THC_ESINGULAR; break; }
    rc = h2d(ctx, ctx->W, hC.data(), PP * sizeof(double)); if (rc) break;
    rc = h2d(ctx, ctx->e, hw.data(), P * sizeof(double)); if (rc) break;
    rc = trsm(ctx, Sl, P, Linv, ctx->W, P, true, tsolve); if (rc) break;   // W = L^-T V

    rc = progress(ctx, "set-up: working basis done, steps", 2, 3); if (rc) break;
    // ---- MP2 guess: M = B^T t_MP2 B with t_MP2 = -(ia|jb)/Delta, T^0 = W^T M W ----
    {
      const int64_t rc0 = std::max<int64_t>(1, std::min<int64_t>(ov, (int64_t)(1.0e9 / (8.0 * ov))));
      double* tb = salloc(rc0 * ov);
      double* tB = salloc(rc0 * P);
      if (!tb || !tB) { ctx->err = "set-up allocation failed"; rc = THC_ENOMEM; break; }
      rc = zero(ctx, tP, PP); if (rc) break;
      for (int64_t r0 = 0; r0 < ov && rc == THC_OK; r0 += rc0) {
        const int64_t rr = std::min(rc0, ov - r0);
        rc = gemm(ctx, mk(rr, ov, nL, ctx->Lov + r0, ov, true, ctx->Lov, ov, false, tb, ov)); if (rc) break;
        MISC(k_mp2_denom(r0, rr, ov, v, ctx->eps, o, tb, s));
        rc = gemm(ctx, mk(rr, P, ov, tb, ov, false, ctx->Bkr, P, false, tB, P)); if (rc) break;
        rc = gemm(ctx, mk(P, P, rr, ctx->Bkr + r0 * P, P, true, tB, P, false, tP, P, 1.0, 1.0)); if (rc) break;
        const int64_t nchunk = (ov + rc0 - 1) / rc0, ci = r0 / rc0 + 1;
        if (nchunk >= 8 && ci % (nchunk / 8) == 0) { rc = progress(ctx, "set-up: MP2 guess, pair rows", r0 + rr, ov); if (rc) break; }
      }
      if (rc) break;
      rc = gemm(ctx, mk(P, P, P, tP, P, false, ctx->W, P, false, Em, P)); if (rc) break;
      rc = gemm(ctx, mk(P, P, P, ctx->W, P, true, Em, P, false, ctx->Th, P)); if (rc) break;
    }
    rc = zero(ctx, ctx->t1, ov); if (rc) break;
    HIPCHK(hipMemcpyAsync(ctx->Th0, ctx->Th, PP * sizeof(double), hipMemcpyDeviceToDevice, s));
    rc = raw_from_basis(ctx, ctx->Th, ctx->Zs); if (rc) break;
    if (Zout) HIPCHK(hipMemcpyAsync(Zout, ctx->Zs, PP * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } while (0);
  sfree();
  if (rc != THC_OK) return rc;
  RCHK(clear_region6(ctx));
  HIPCHK(hipStreamSynchronize(s));
  ctx->built = true;
  ctx->guess_pending = true;
  ctx->have_last = false;
  ctx->diis_n = 0;
  ctx->diis_head = 0;
  return THC_OK;
}

int thc_mp2_density(thc_ctx* ctx, const double* Z, double* Doo, double* Dvv) {
  if (!ctx) return THC_EINVAL;
  RCHK(need_built(ctx));
  if (!Doo || !Dvv) { ctx->err = "null output"; return THC_EINVAL; }
  hipStream_t s = ctx->stream;
  const int64_t o = ctx->o, v = ctx->v, P = ctx->P, PP = P * P;
  const double *Yo = ctx->Yo, *Yv = ctx->Yv, *Go = ctx->Go, *Gv = ctx->Gv;
  const double* T = Z ? Z : ctx->Zs;
  // T S T with S = o o v (the metric, Eq. 51-52)
  RCHK(gemm(ctx, mk(P, P, P, ctx->S, P, false, T, P, false, ctx->Qm, P)));
  RCHK(gemm(ctx, mk(P, P, P, T, P, false, ctx->Qm, P, false, ctx->E9, P)));
  // Coulomb-like parts (Eq. 53, 54): D_oo = -4 Yo (v o TST) Yo^T, D_vv = 4 Yv (o o TST) Yv^T
  MISC(k_hadamard(PP, Gv, ctx->E9, 1.0, 0.0, ctx->ot, s));
  MISC(k_hadamard(PP, Go, ctx->E9, 1.0, 0.0, ctx->vt, s));
  RCHK(gemm(ctx, mk(o, P, P, Yo, P, false, ctx->ot, P, false, ctx->tmpoP, P)));
  RCHK(gemm(ctx, mk(o, o, P, ctx->tmpoP, P, false, Yo, P, true, Doo, o, -4.0, 0.0)));
  RCHK(gemm(ctx, mk(v, P, P, Yv, P, false, ctx->vt, P, false, ctx->tmpvP, P)));
  RCHK(gemm(ctx, mk(v, v, P, ctx->tmpvP, P, false, Yv, P, true, Dvv, v, 4.0, 0.0)));
  // Exchange-like parts (Eq. 55, 56), for blocks of the outer index r (i, or a):
  //   M_r = (T^T diag(y_r) G1) o G2,  K_r = M_r T,  u_r^Y = sum_X G1^XY K_r^XY,
  //   D[r][s] += f sum_Y y_s^Y u_r^Y
  // with (G1, G2, y, f) = (v, o, y_o, 2) for D_oo and (o, v, y_v, -2) for D_vv.
  const int64_t ch = std::min(ctx->nb, ctx->nL);  // blocks fit the fused pass's nb x P^2 buffers
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t n = pass == 0 ? o : v;
    const double* Yr = pass == 0 ? Yo : Yv;
    const double *G1 = pass == 0 ? Gv : Go, *G2 = pass == 0 ? Go : Gv;
    double* D = pass == 0 ? Doo : Dvv;
    const double f = pass == 0 ? 2.0 : -2.0;
    for (int64_t r0 = 0; r0 < n; r0 += ch) {
      const int64_t nr = std::min(ch, n - r0);
      Gemm g = batched(mk(P, P, P, T, P, true, G1, P, false, ctx->Ccat, P), nr, 0, 0, PP);
      g.kscaleA = Yr + r0 * P; g.ksA = 1; g.sksA = P;
      g.hmul = G2; g.ldh = P;
      RCHK(gemm(ctx, g));
      RCHK(gemm(ctx, batched(mk(P, P, P, ctx->Ccat, P, false, T, P, false, ctx->Dcat, P), nr, PP, 0, PP)));
      MISC(k_colsum_rowscaled(nr, P, P, G1, ctx->Dcat, PP, ctx->Dt, nr, s));
      RCHK(gemm(ctx, mk(nr, n, P, ctx->Dt, nr, true, Yr, P, true, D + r0 * n, n, f, 1.0)));
    }
  }
  return THC_OK;
}

int thc_residual_terms(thc_ctx* ctx, const double* Z, const double* t1, uint32_t mask, double* sigma, double* sigma1) {
  if (!ctx) return THC_EINVAL;
  RCHK(need_built(ctx));
  if (!Z || !sigma) { ctx->err = "null argument"; return THC_EINVAL; }
  ctx->want_mixed = ctx->opt.precision >= 1;
  RCHK(residual_impl(ctx, Z, ctx->opt.singles ? t1 : nullptr, mask));
  HIPCHK(hipMemcpyAsync(sigma, ctx->sig, ctx->P * ctx->P * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (sigma1) HIPCHK(hipMemcpyAsync(sigma1, ctx->sig1, ctx->ov * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return THC_OK;
}

int thc_residual(thc_ctx* ctx, const double* Z, const double* t1, double* sigma, double* sigma1, double* norms) {
  if (!ctx) return THC_EINVAL;
  RCHK(thc_residual_terms(ctx, Z, t1, THC_TERM_ALL, sigma, sigma1));
  if (norms) {
    RCHK(project_basis(ctx));
    double h[10];
    RCHK(d2h(ctx, h, ctx->scal, 10 * sizeof(double)));
    norms[0] = std::sqrt(h[8]);
    norms[1] = std::sqrt(h[9]);
    RCHK(check_finite_host(ctx, norms, 2, "residual norms"));
  }
  return THC_OK;
}

int thc_energy(thc_ctx* ctx, double* e_corr) {
  if (!ctx || !e_corr) return THC_EINVAL;
  RCHK(need_built(ctx));
  ctx->want_mixed = false;
  RCHK(residual_impl(ctx, ctx->Zs, ctx->t1, 0u));
  double h[4];
  RCHK(read_scalars(ctx, h, 4));
  *e_corr = energy_from_scalars(h, ctx->opt.singles != 0);
  RCHK(check_finite_host(ctx, e_corr, 1, "energy"));
  return THC_OK;
}

int thc_get_state(thc_ctx* ctx, double* Z, double* t1) {
  if (!ctx) return THC_EINVAL;
  RCHK(need_built(ctx));
  if (Z) HIPCHK(hipMemcpyAsync(Z, ctx->Zs, ctx->P * ctx->P * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (t1) HIPCHK(hipMemcpyAsync(t1, ctx->t1, ctx->ov * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return THC_OK;
}

int thc_set_state(thc_ctx* ctx, const double* Z, const double* t1) {
  if (!ctx || !Z) return THC_EINVAL;
  RCHK(need_built(ctx));
  HIPCHK(hipMemcpyAsync(ctx->Zs, Z, ctx->P * ctx->P * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (t1 && ctx->opt.singles)
    HIPCHK(hipMemcpyAsync(ctx->t1, t1, ctx->ov * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  else
    RCHK(zero(ctx, ctx->t1, ctx->ov));
  RCHK(basis_from_raw(ctx, ctx->Zs, ctx->Th));
  ctx->diis_n = 0;
  ctx->diis_head = 0;
  ctx->guess_pending = false;
  ctx->have_last = false;
  return THC_OK;
}

// Checkpoint: a fixed header, then T^ [P][P], t1 [ov], delta [P], the DIIS vectors and errors
// [dm][P P + ov] each and the error overlap matrix [dm][dm], as raw FP64.
namespace {
struct CkptHeader {
  char magic[8];
  int64_t P, ov, dm, diis_n, diis_head, has_shift, have_last;
  double E_last;
};
constexpr char CKPT_MAGIC[8] = {'T', 'H', 'C', 'C', 'K', 'P', 'T', '1'};
size_t ckpt_doubles(const thc_ctx* ctx) {
  const int64_t P = ctx->P, ov = ctx->ov, dm = ctx->opt.diis_max, len = P * P + ov;
  return (size_t)(P * P + ov + P + 2 * dm * len + dm * dm);
}
}  // namespace

int thc_checkpoint_bytes(thc_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return THC_EINVAL;
  RCHK(need_built(ctx));
  *bytes = sizeof(CkptHeader) + 8 * ckpt_doubles(ctx);
  return THC_OK;
}

int thc_save_checkpoint(thc_ctx* ctx, void* host, size_t bytes) {
  if (!ctx || !host) return THC_EINVAL;
  RCHK(need_built(ctx));
  const int64_t P = ctx->P, ov = ctx->ov, dm = ctx->opt.diis_max, len = P * P + ov;
  if (bytes < sizeof(CkptHeader) + 8 * ckpt_doubles(ctx)) {
    ctx->err = "checkpoint buffer too small (thc_checkpoint_bytes)";
    return THC_EINVAL;
  }
  CkptHeader h{};
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.P = P; h.ov = ov; h.dm = dm; h.diis_n = ctx->diis_n; h.diis_head = ctx->diis_head;
  h.has_shift = ctx->has_shift ? 1 : 0; h.have_last = ctx->have_last ? 1 : 0; h.E_last = ctx->E_last;
  std::memcpy(host, &h, sizeof h);
  double* d = reinterpret_cast<double*>(static_cast<char*>(host) + sizeof h);
  RCHK(d2h(ctx, d, ctx->Th, P * P * sizeof(double)));
  RCHK(d2h(ctx, d + P * P, ctx->t1, ov * sizeof(double)));
  RCHK(d2h(ctx, d + P * P + ov, ctx->delta, P * sizeof(double)));
  if (dm > 0) {
    RCHK(d2h(ctx, d + P * P + ov + P, ctx->dvec, dm * len * sizeof(double)));
    RCHK(d2h(ctx, d + P * P + ov + P + dm * len, ctx->derr, dm * len * sizeof(double)));
    std::memcpy(d + P * P + ov + P + 2 * dm * len, ctx->diisB.data(), (size_t)(dm * dm) * sizeof(double));
  }
  return THC_OK;
}

int thc_load_checkpoint(thc_ctx* ctx, const void* host, size_t bytes) {
  if (!ctx || !host) return THC_EINVAL;
  RCHK(need_built(ctx));
  const int64_t P = ctx->P, ov = ctx->ov, dm = ctx->opt.diis_max, len = P * P + ov;
  CkptHeader h;
  if (bytes < sizeof h) return THC_EINVAL;
  std::memcpy(&h, host, sizeof h);
  if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.P != P || h.ov != ov || h.dm != dm ||
      bytes < sizeof h + 8 * ckpt_doubles(ctx) || h.diis_n < 0 || h.diis_n > dm || h.diis_head < 0 ||
      (dm > 0 && h.diis_head >= dm)) {
    ctx->err = "not a checkpoint of a context with these sizes and DIIS subspace";
    return THC_EINVAL;
  }
  const double* d = reinterpret_cast<const double*>(static_cast<const char*>(host) + sizeof h);
  RCHK(h2d(ctx, ctx->Th, d, P * P * sizeof(double)));
  RCHK(h2d(ctx, ctx->t1, d + P * P, ov * sizeof(double)));
  RCHK(h2d(ctx, ctx->delta, d + P * P + ov, P * sizeof(double)));
  if (dm > 0) {
    RCHK(h2d(ctx, ctx->dvec, d + P * P + ov + P, dm * len * sizeof(double)));
    RCHK(h2d(ctx, ctx->derr, d + P * P + ov + P + dm * len, dm * len * sizeof(double)));
    std::memcpy(ctx->diisB.data(), d + P * P + ov + P + 2 * dm * len, (size_t)(dm * dm) * sizeof(double));
  }
  RCHK(raw_from_basis(ctx, ctx->Th, ctx->Zs));
  ctx->has_shift = h.has_shift != 0;
  ctx->diis_n = (int)h.diis_n;
  ctx->diis_head = (int)h.diis_head;
  ctx->E_last = h.E_last;
  ctx->have_last = h.have_last != 0;
  ctx->guess_pending = false;
  return THC_OK;
}

int thc_iterate(thc_ctx* ctx, double tol, int maxit, int* iters, double* rnorm) {
  if (!ctx || maxit < 1 || !(tol >= 0.0)) return THC_EINVAL;
  RCHK(need_built(ctx));
  hipStream_t s = ctx->stream;
  const int64_t P = ctx->P, PP = P * P, ov = ctx->ov, len = PP + ov;
  const bool singles = ctx->opt.singles != 0;
  const int dm = ctx->opt.diis_max;
  // a call continues the previous one's iteration: its first energy is compared with the last
  // one (unless the state was set from outside since)
  double E_old = ctx->E_last;
  bool have_old = ctx->have_last;
  ctx->hist_e.clear();
  ctx->hist_r.clear();
  ctx->hist_t.clear();
  const auto t_start = std::chrono::steady_clock::now();
  // precision ladder (mixed precision): reduced-precision residuals until their norm has dropped
  // 1e4-fold, is within 10 tol, stops decreasing, or is predicted below tol for the next iteration;
  // then FP64 residuals, which alone may declare convergence
  bool mixed_phase = ctx->opt.precision >= 1;
  double rn_first = -1.0, rn_prev = 0.0;
  int mixed_its = 0;
  ctx->hist_mixed.clear();
  ctx->hist_flags.clear();
  // divergence: a residual norm that is not finite, above 10 times the smallest of this run, or
  // larger than its predecessor three times in a row.  The first time, the solver restarts from
  // the MP2 guess with the plain denominators e_P + e_Q and an empty DIIS subspace; the second
  // time it stops with THC_EDIVERGED.
  double rn_min = -1.0, rn_last = -1.0;
  int rises = 0;
  bool fell_back = false, restarted = false;
  // learned start (thc_options.guess = 1): the network's prediction from the features of the MP2
  // guess scales the start and shifts the denominators; the divergence restart above is its fallback
  bool learned = false;
  int learned_its = 0;
  double rn_learned = 0.0;
  if (ctx->opt.guess == 1 && ctx->guess_pending) {
    thc_mlp* net = ctx->guess_net;
    if (!net) {
      ctx->err = "thc_options.guess = 1 needs a network (thc_set_guess_network)";
      return THC_ESTATE;
    }
    if (12 * P * (int64_t)sizeof(float) > len * (int64_t)sizeof(double)) {
      ctx->err = "the learned start needs nP^2 + o v >= 6 nP";
      return THC_EINVAL;
    }
    float* phi = (float*)ctx->dT;  // the Jacobi step's buffer is free before the first residual
    float* pred = phi + P * 10;
    MISC(k_dot(PP, ctx->Th, ctx->Th, ctx->scal + 40, s));
    MISC(k_guess_features(P, ctx->o, ctx->v, ctx->Th, ctx->e, ctx->eps, ctx->scal + 40, phi, s));
    if (hipStreamSynchronize(net->stream) != hipSuccess) return THC_EDEVICE;  // its parameters are final
    if (!net->packed) {
      HIPCHK(mlp_pack_bf16(net->n_in, net->n_out, net->p, net->wb, net->bb, s));
      net->packed = true;
    }
    HIPCHK(mlp_infer_bf16(P, net->n_in, net->n_out, phi, net->mu_in, net->sd_in, net->wb, net->bb, net->mu_out,
                          net->sd_out, pred, s));
    MISC(k_guess_apply(P, pred, net->n_out, ctx->Th, ctx->delta, s));
    ctx->has_shift = net->n_out > 1;
    RCHK(raw_from_basis(ctx, ctx->Th, ctx->Zs));
    ctx->diis_n = 0;
    ctx->diis_head = 0;
    learned = true;
    have_old = ctx->have_last = false;
  }
  ctx->guess_pending = false;
  for (int it = 1; it <= maxit; ++it) {
    ctx->want_mixed = mixed_phase;
    RCHK(residual_impl(ctx, ctx->Zs, singles ? ctx->t1 : nullptr, THC_TERM_ALL));
    RCHK(project_basis(ctx));
    double h[10];
    RCHK(read_scalars(ctx, h, 10));
    const double E = energy_from_scalars(h, singles);
    const double rn = std::sqrt(h[8] + h[9]);
    const bool finite = std::isfinite(E) && std::isfinite(rn);
    if (iters) *iters = it;
    if (rnorm) *rnorm = rn;
    ctx->hist_e.push_back(E);
    ctx->hist_r.push_back(rn);
    ctx->hist_t.push_back(std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
    ctx->hist_mixed.push_back(mixed_phase ? 1 : 0);
    ctx->hist_flags.push_back((mixed_phase ? THC_ITER_MIXED : 0) | (restarted ? THC_ITER_RESTARTED : 0) |
                              (learned ? THC_ITER_LEARNED : 0));
    restarted = false;
    if (finite && rn_last >= 0.0) rises = rn > rn_last ? rises + 1 : 0;
    // a learned start that has not cut the residual norm tenfold in three iterations is abandoned
    // like a divergent one (from the MP2 guess the norm falls by orders of magnitude in that time)
    if (learned && ++learned_its == 1) rn_learned = rn;
    const bool stalled = learned && learned_its == 3 && !(rn < 0.1 * rn_learned);
    const bool diverged = !finite || (rn_min > 0.0 && rn > 10.0 * rn_min) || rises >= 3 || stalled;
    if (finite) {
      rn_last = rn;
      rn_min = rn_min < 0.0 ? rn : std::min(rn_min, rn);
    }
    if (diverged) {
      if (fell_back) {
        ctx->err = finite ? "the iteration diverged again after restarting from the MP2 guess"
                          : "residual or energy is not finite after restarting from the MP2 guess";
        return THC_EDIVERGED;
      }
      fell_back = restarted = true;
      learned = false;
      ctx->have_last = false;
      HIPCHK(hipMemcpyAsync(ctx->Th, ctx->Th0, PP * sizeof(double), hipMemcpyDeviceToDevice, s));
      RCHK(zero(ctx, ctx->t1, ov));
      RCHK(raw_from_basis(ctx, ctx->Th, ctx->Zs));
      ctx->has_shift = false;
      ctx->diis_n = 0;
      ctx->diis_head = 0;
      mixed_phase = ctx->opt.precision >= 1;
      rn_first = -1.0;
      mixed_its = 0;
      rn_min = rn_last = -1.0;
      rises = 0;
      have_old = false;
      continue;
    }
    if (mixed_phase) {
      ++mixed_its;
      if (rn_first < 0.0) rn_first = rn;
      // FP64 from the next iteration on once the norm has dropped 1e4-fold, is within 10 tol, has
      // stopped decreasing, or falls fast enough that the next one is predicted below tol (then
      // that iteration can already declare convergence)
      const bool next_below_tol = mixed_its >= 2 && rn_prev > 0.0 && rn * (rn / rn_prev) < tol;
      if (rn < 1e-4 * rn_first || rn < 10.0 * tol || next_below_tol || (mixed_its >= 3 && rn > 0.7 * rn_prev))
        mixed_phase = false;
      rn_prev = rn;
    } else if (have_old && rn < tol && std::fabs(E - E_old) < ctx->opt.tol_energy) {
      ctx->E_last = E;
      ctx->have_last = true;
      return THC_OK;
    }
    E_old = E;
    have_old = true;
    ctx->E_last = E;
    ctx->have_last = true;
    // Jacobi step in the working basis; (dT, dt1) is the DIIS error vector
    double* dTp = ctx->dT;
    double* dt1p = ctx->dT + PP;
    MISC(k_jacobi(P, ctx->o, ctx->v, ctx->sigh, ctx->e, ctx->has_shift ? ctx->delta : nullptr,
                  singles ? ctx->sig1 : nullptr, ctx->eps, ctx->Th, ctx->t1,
                  dTp, dt1p, s));
    if (dm > 0) {
      const int slot = ctx->diis_head;
      double* vs = ctx->dvec + (int64_t)slot * len;
      double* es = ctx->derr + (int64_t)slot * len;
      HIPCHK(hipMemcpyAsync(vs, ctx->Th, PP * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(vs + PP, ctx->t1, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(es, ctx->dT, len * sizeof(double), hipMemcpyDeviceToDevice, s));
      ctx->diis_head = (slot + 1) % dm;
      if (ctx->diis_n < dm) ctx->diis_n++;
      const int mfull = ctx->diis_n;
      // inner products of the new error with every stored error (device), B on the host
      std::vector<int> slots(mfull);
      for (int k = 0; k < mfull; ++k) slots[k] = (ctx->diis_head - mfull + k + 2 * dm) % dm;  // oldest first
      for (int k = 0; k < mfull; ++k)
        MISC(k_dot(len, ctx->derr + (int64_t)slots[k] * len, es, ctx->scal + 16 + k, s));
      double bd[16];
      RCHK(d2h(ctx, bd, ctx->scal + 16, mfull * sizeof(double)));
      for (int k = 0; k < mfull; ++k) {
        ctx->diisB[(size_t)slots[k] * dm + slot] = bd[k];
        ctx->diisB[(size_t)slot * dm + slots[k]] = bd[k];
      }
      // conditioning: while the error overlap matrix of the kept vectors has a condition number
      // above 1e12, the oldest vector is dropped
      int m = ctx->diis_n;
      while (m >= 2) {
        std::vector<double> Bm((size_t)m * m), wv(m);
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < m; ++j)
            Bm[(size_t)i * m + j] = ctx->diisB[(size_t)slots[mfull - m + i] * dm + slots[mfull - m + j]];
        if (host_syev(m, Bm.data(), wv.data()) == 0 && wv[0] > 1e-12 * wv[m - 1]) break;
        --m;
        ctx->hist_flags.back() |= THC_ITER_DIIS_DROPPED;
      }
      ctx->diis_n = m;
      if (m < mfull) slots.erase(slots.begin(), slots.begin() + (mfull - m));
      if (m >= 2) {
        // Pulay: [B -1; -1 0] [c; l] = [0; -1], solved by Gaussian elimination with pivoting
        const int N = m + 1;
        std::vector<double> A((size_t)N * N), b(N, 0.0);
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < m; ++j) A[(size_t)i * N + j] = ctx->diisB[(size_t)slots[i] * dm + slots[j]];
        for (int i = 0; i < m; ++i) { A[(size_t)i * N + m] = -1.0; A[(size_t)m * N + i] = -1.0; }
        A[(size_t)m * N + m] = 0.0;
        b[m] = -1.0;
        bool ok = true;
        for (int c = 0; c < N && ok; ++c) {
          int piv = c;
          for (int r = c + 1; r < N; ++r)
            if (std::fabs(A[(size_t)r * N + c]) > std::fabs(A[(size_t)piv * N + c])) piv = r;
          if (std::fabs(A[(size_t)piv * N + c]) < 1e-300) { ok = false; break; }
          if (piv != c) {
            for (int k = 0; k < N; ++k) std::swap(A[(size_t)c * N + k], A[(size_t)piv * N + k]);
            std::swap(b[c], b[piv]);
          }
          for (int r = c + 1; r < N; ++r) {
            const double f = A[(size_t)r * N + c] / A[(size_t)c * N + c];
            for (int k = c; k < N; ++k) A[(size_t)r * N + k] -= f * A[(size_t)c * N + k];
            b[r] -= f * b[c];
          }
        }
        std::vector<double> x(N, 0.0);
        if (ok) {
          for (int r = N - 1; r >= 0; --r) {
            double acc = b[r];
            for (int k = r + 1; k < N; ++k) acc -= A[(size_t)r * N + k] * x[k];
            x[r] = acc / A[(size_t)r * N + r];
          }
          for (int k = 0; k < m; ++k) ok = ok && std::isfinite(x[k]);
        }
        if (ok) {
          std::vector<const double*> vecs(m);
          for (int k = 0; k < m; ++k) vecs[k] = ctx->dvec + (int64_t)slots[k] * len;
          // extrapolate into the first work vector, then split into Th / t1
          MISC(k_lincomb(len, m, x.data(), vecs.data(), ctx->dT, s));
          HIPCHK(hipMemcpyAsync(ctx->Th, ctx->dT, PP * sizeof(double), hipMemcpyDeviceToDevice, s));
          HIPCHK(hipMemcpyAsync(ctx->t1, ctx->dT + PP, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
      }
    }
    RCHK(raw_from_basis(ctx, ctx->Th, ctx->Zs));
  }
  ctx->err = "iteration limit reached";
  return THC_ENOTCONV;
}

int thc_history_flags(const thc_ctx* ctx, int max, int* flags, int* count) {
  if (!ctx || max < 0 || (max > 0 && !flags)) return THC_EINVAL;
  const int n = (int)ctx->hist_flags.size();
  for (int k = 0; k < std::min(n, max); ++k) flags[k] = ctx->hist_flags[k];
  if (count) *count = n;
  return THC_OK;
}

int thc_history_precision(const thc_ctx* ctx, int max, int* mixed, int* count) {
  if (!ctx || max < 0 || (max > 0 && !mixed)) return THC_EINVAL;
  const int n = (int)ctx->hist_mixed.size();
  for (int k = 0; k < std::min(n, max); ++k) mixed[k] = ctx->hist_mixed[k];
  if (count) *count = n;
  return THC_OK;
}

int thc_history(const thc_ctx* ctx, int max, double* energy, double* rnorm, double* seconds, int* count) {
  if (!ctx || max < 0) return THC_EINVAL;
  const int n = (int)ctx->hist_e.size();
  const int m = std::min(n, max);
  for (int i = 0; i < m; ++i) {
    if (energy) energy[i] = ctx->hist_e[i];
    if (rnorm) rnorm[i] = ctx->hist_r[i];
    if (seconds) seconds[i] = ctx->hist_t[i];
  }
  if (count) *count = n;
  return THC_OK;
}

int thc_memory_bytes(const thc_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return THC_EINVAL;
  *bytes = ctx->bytes;
  return THC_OK;
}

int thc_plan(const thc_ctx* ctx, thc_plan_info* out) {
  if (!ctx || !out) return THC_EINVAL;
  if (!ctx->built) return THC_ESTATE;
  fill_plan_info(ctx, ctx->hfilled, ctx->nhtiles, ctx->hslots, (double)ctx->bytes, out);
  return THC_OK;
}

int thc_profile(thc_ctx* ctx, int enable) {
  if (!ctx) return THC_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return THC_EDEVICE;
  ctx->prof = enable != 0;
  ctx->recs.clear();
  ctx->pool_used = 0;
  ctx->gemm_flops = ctx->gemm_flops32 = ctx->gemm_flops16 = 0.0;
  return THC_OK;
}

int thc_profile_get(thc_ctx* ctx, const char* name, double* total_ms, int64_t* launches) {
  if (!ctx || !name) return THC_EINVAL;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : ctx->recs) {
    if (r.name != name) continue;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    cnt += r.launches;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return THC_OK;
}

int thc_profile_flops(const thc_ctx* ctx, double* fp64_flops, double* fp32_flops, double* bf16x3_flops) {
  if (!ctx) return THC_EINVAL;
  if (fp64_flops) *fp64_flops = ctx->gemm_flops;
  if (fp32_flops) *fp32_flops = ctx->gemm_flops32;
  if (bf16x3_flops) *bf16x3_flops = ctx->gemm_flops16;
  return THC_OK;
}

// ------------------------------------------------------------------------------------------
// Weighted CP-ALS (Sec. II.c-d, Eq. 15-16, 21; Appendix I, Eq. 43-46).
namespace {
struct CpWork {
  std::vector<void*> mem;
  ~CpWork() { for (void* q : mem) (void)hipFree(q); }
  double* get(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(double)) != hipSuccess) return nullptr;
    mem.push_back(q);
    return (double*)q;
  }
};

#define CPCHK(expr)                        \
  do {                                     \
    if ((expr) != hipSuccess) return THC_EDEVICE; \
  } while (0)

// Solves S U = B ([n][m], column c one right-hand side) by conjugate gradients preconditioned with
// diag(S), from the U given; stops when every column's residual is below tol times its right-hand
// side.  *iters: iterations taken; returns THC_ENOTCONV if maxit is reached first.
int cp_pcg(int64_t n, int64_t m, const double* S, const double* B, double* U, double tol, int maxit, double* d,
           double* R, double* Zr, double* P, double* Q, double* rz, double* rz2, double* pq, double* rr, double* bb,
           int* iters, hipStream_t s) {
  CPCHK(cp_diag(n, S, d, s));
  CPCHK(hipMemcpyAsync(R, B, n * m * sizeof(double), hipMemcpyDeviceToDevice, s));
  CPCHK(gemm_f64(mk(n, m, n, S, n, false, U, m, false, R, m, -1.0, 1.0), s));
  CPCHK(cp_cg_precond(n, m, d, R, Zr, s));
  CPCHK(hipMemcpyAsync(P, Zr, n * m * sizeof(double), hipMemcpyDeviceToDevice, s));
  CPCHK(cp_col_dot(n, m, R, Zr, rz, s));
  CPCHK(cp_col_dot(n, m, B, B, bb, s));
  std::vector<double> hr(m), hb(m);
  CPCHK(hipMemcpyAsync(hb.data(), bb, m * sizeof(double), hipMemcpyDeviceToHost, s));
  CPCHK(hipStreamSynchronize(s));
  for (int it = 1; it <= maxit; ++it) {
    CPCHK(gemm_f64(mk(n, m, n, S, n, false, P, m, false, Q, m), s));
    CPCHK(cp_col_dot(n, m, P, Q, pq, s));
    CPCHK(cp_cg_step(n, m, rz, pq, P, Q, U, R, s));
    CPCHK(cp_col_dot(n, m, R, R, rr, s));
    CPCHK(hipMemcpyAsync(hr.data(), rr, m * sizeof(double), hipMemcpyDeviceToHost, s));
    CPCHK(hipStreamSynchronize(s));
    bool done = true;
    for (int64_t c = 0; c < m && done; ++c) done = std::sqrt(hr[c]) <= tol * std::sqrt(hb[c]);
    *iters = it;
    if (done) return THC_OK;
    CPCHK(cp_cg_precond(n, m, d, R, Zr, s));
    CPCHK(cp_col_dot(n, m, R, Zr, rz2, s));
    CPCHK(cp_cg_dir(n, m, rz2, rz, Zr, P, s));
    std::swap(rz, rz2);
  }
  return THC_ENOTCONV;
}
}  // namespace

int thc_cp_als(const double* A, int64_t I, int64_t J, int64_t K, int64_t n, const double* w1, const double* w2,
               const double* w3, double* X, double* Y, double* Z, int sweeps, double cg_tol, int cg_maxit,
               double* objective, int* cg_iters, void* stream) {
  if (!A || !X || !Y || !Z || I < 1 || J < 1 || K < 1 || n < 1 || sweeps < 0 || !(cg_tol > 0.0) || cg_maxit < 1)
    return THC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t m = std::max(std::max(I, J), K), IJ = I * J;
  CpWork w;
  double *TB = w.get(IJ * n), *Xw = w.get(I * n), *Yw = w.get(J * n), *Zw = w.get(K * n), *Zwt = w.get(K * n);
  double *G1 = w.get(n * n), *G2 = w.get(n * n), *G3 = w.get(n * n), *S = w.get(n * n), *H = w.get(n * n);
  double *Bt = w.get(n * m), *U = w.get(n * m), *R = w.get(n * m), *Zr = w.get(n * m), *P = w.get(n * m),
         *Qb = w.get(n * m);
  double *d = w.get(n), *rz = w.get(m), *rz2 = w.get(m), *pq = w.get(m), *rr = w.get(m), *bb = w.get(m);
  const int64_t nparts = cp_wnorm2_parts(I, J, K);
  double *parts = w.get(nparts), *sc = w.get(4);
  if (!TB || !Xw || !Yw || !Zw || !Zwt || !G1 || !G2 || !G3 || !S || !H || !Bt || !U || !R || !Zr || !P || !Qb || !d ||
      !rz || !rz2 || !pq || !rr || !bb || !parts || !sc)
    return THC_ENOMEM;
  int worst = 0, rc_all = THC_OK;
  // one factor update: S U = B with U = F^T warm-started from F, then F = U^T
  auto solve = [&](double* F, int64_t rows) -> int {
    CPCHK(k_copy2d(1, n, rows, F, n, 0, U, rows, 0, true, s));
    int its = 0;
    const int rc = cp_pcg(n, rows, S, Bt, U, cg_tol, cg_maxit, d, R, Zr, P, Qb, rz, rz2, pq, rr, bb, &its, s);
    worst = std::max(worst, its);
    if (rc == THC_ENOTCONV) rc_all = THC_ENOTCONV;
    else if (rc != THC_OK) return rc;
    CPCHK(k_copy2d(1, rows, n, U, rows, 0, F, n, 0, true, s));
    return THC_OK;
  };
  // objective = |A_w|^2 - 2 sum_kn w3_k^2 Z_kn R_Z[k][n] + sum (G1 o G2 o G3), all with the current factors
  double anorm = 0.0;
  {
    CPCHK(cp_wnorm2(I, J, K, A, w1, w2, w3, parts, s));
    CPCHK(k_sum(nparts, parts, sc, s));
    CPCHK(hipMemcpyAsync(&anorm, sc, sizeof(double), hipMemcpyDeviceToHost, s));
    CPCHK(hipStreamSynchronize(s));
  }
  auto grams = [&]() -> int {  // Xw, Yw, Zw and G1 = X^T Xw, G2 = Y^T Yw, G3 = Z^T Zw
    CPCHK(cp_weighted_rows(I, n, w1, X, Xw, s));
    CPCHK(cp_weighted_rows(J, n, w2, Y, Yw, s));
    CPCHK(cp_weighted_rows(K, n, w3, Z, Zw, s));
    CPCHK(gemm_f64(mk(n, n, I, X, n, true, Xw, n, false, G1, n), s));
    CPCHK(gemm_f64(mk(n, n, J, Y, n, true, Yw, n, false, G2, n), s));
    CPCHK(gemm_f64(mk(n, n, K, Z, n, true, Zw, n, false, G3, n), s));
    return THC_OK;
  };
  auto record = [&](int idx) -> int {  // objective of the current factors into objective[idx]
    if (!objective) return THC_OK;
    RCHK(grams());
    // R_Z^T = KR(Xw, Yw)^T A  ([n][K])
    CPCHK(k_kr(I, J, n, Xw, Yw, TB, s));
    CPCHK(gemm_f64(mk(n, K, IJ, TB, n, true, A, K, false, Bt, K), s));
    CPCHK(k_copy2d(1, n, K, Zw, n, 0, Zwt, K, 0, true, s));
    CPCHK(k_dot(n * K, Zwt, Bt, sc, s));
    CPCHK(k_hadamard(n * n, G1, G2, 1.0, 0.0, H, s));
    CPCHK(k_dot(n * n, H, G3, sc + 1, s));
    double h[2];
    CPCHK(hipMemcpyAsync(h, sc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    CPCHK(hipStreamSynchronize(s));
    objective[idx] = anorm - 2.0 * h[0] + h[1];
    return THC_OK;
  };
  RCHK(record(0));
  for (int sw = 0; sw < sweeps; ++sw) {
    RCHK(grams());
    // X: T = A (W3^2 Z) (IJ x n); B_X^T[n][i] = sum_j w2_j^2 Y_jn T[i][j][n]; S = G2 o G3
    CPCHK(gemm_f64(mk(IJ, n, K, A, K, false, Zw, n, false, TB, n), s));
    CPCHK(cp_mttkrp_reduce(I, J, n, TB, Yw, true, Bt, s));
    CPCHK(k_hadamard(n * n, G2, G3, 1.0, 0.0, S, s));
    RCHK(solve(X, I));
    // Y: B_Y^T[n][j] = sum_i w1_i^2 X_in T[i][j][n] (T unchanged: it depends on Z only); S = G1 o G3
    CPCHK(cp_weighted_rows(I, n, w1, X, Xw, s));
    CPCHK(gemm_f64(mk(n, n, I, X, n, true, Xw, n, false, G1, n), s));
    CPCHK(cp_mttkrp_reduce(I, J, n, TB, Xw, false, Bt, s));
    CPCHK(k_hadamard(n * n, G1, G3, 1.0, 0.0, S, s));
    RCHK(solve(Y, J));
    // Z: B_Z^T = KR(W1^2 X, W2^2 Y)^T A ([n][K]); S = G1 o G2
    CPCHK(cp_weighted_rows(J, n, w2, Y, Yw, s));
    CPCHK(gemm_f64(mk(n, n, J, Y, n, true, Yw, n, false, G2, n), s));
    CPCHK(k_kr(I, J, n, Xw, Yw, TB, s));
    CPCHK(gemm_f64(mk(n, K, IJ, TB, n, true, A, K, false, Bt, K), s));
    CPCHK(k_hadamard(n * n, G1, G2, 1.0, 0.0, S, s));
    RCHK(solve(Z, K));
    RCHK(record(sw + 1));
  }
  CPCHK(hipStreamSynchronize(s));
  if (cg_iters) *cg_iters = worst;
  return rc_all;
}

int thc_dgemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc, int64_t sC,
              int64_t batch, void* stream) {
  if (M < 0 || N < 0 || K < 0 || batch < 0 || sA < 0 || sB < 0 || sC < 0) return THC_EINVAL;
  if (M == 0 || N == 0 || batch == 0) return THC_OK;  // nothing to compute
  // every row of op(A), op(B) and C within its leading dimension, and the operands present
  if (!C || ldc < N || (K > 0 && (!A || !B || lda < (transA ? M : K) || ldb < (transB ? K : N))))
    return THC_EINVAL;
  Gemm g = batched(mk(M, N, K, A, lda, transA != 0, B, ldb, transB != 0, C, ldc, alpha, beta), batch, sA, sB, sC);
  if (gemm_f64(g, (hipStream_t)stream) != hipSuccess) return THC_EDEVICE;
  return THC_OK;
}

// ------------------------------------------------------------------------------------------
// Learned starting guess (not part of the paper): features, application, Jacobi shift, state in
// the working basis and least-squares training targets.

int thc_guess_features(thc_ctx* ctx, float* phi) {
  if (!ctx || !phi) return THC_EINVAL;
  RCHK(need_built(ctx));
  MISC(k_dot(ctx->P * ctx->P, ctx->Th, ctx->Th, ctx->scal + 40, ctx->stream));
  MISC(k_guess_features(ctx->P, ctx->o, ctx->v, ctx->Th, ctx->e, ctx->eps, ctx->scal + 40, phi, ctx->stream));
  return THC_OK;
}

int thc_guess_apply(thc_ctx* ctx, const float* pred, int64_t ld) {
  if (!ctx || !pred || ld < 1) return THC_EINVAL;
  RCHK(need_built(ctx));
  ctx->guess_pending = false;
  ctx->have_last = false;
  MISC(k_guess_apply(ctx->P, pred, ld, ctx->Th, ctx->delta, ctx->stream));
  ctx->has_shift = ld > 1;
  RCHK(raw_from_basis(ctx, ctx->Th, ctx->Zs));
  ctx->diis_n = 0;
  ctx->diis_head = 0;
  return THC_OK;
}

int thc_set_shift(thc_ctx* ctx, const double* delta) {
  if (!ctx) return THC_EINVAL;
  RCHK(need_built(ctx));
  ctx->guess_pending = false;
  ctx->have_last = false;
  if (delta) HIPCHK(hipMemcpyAsync(ctx->delta, delta, ctx->P * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  ctx->has_shift = delta != nullptr;
  ctx->diis_n = 0;
  ctx->diis_head = 0;
  return THC_OK;
}

int thc_working(thc_ctx* ctx, double* Th, double* sigma_hat) {
  if (!ctx) return THC_EINVAL;
  RCHK(need_built(ctx));
  const int64_t PP = ctx->P * ctx->P;
  if (Th) HIPCHK(hipMemcpyAsync(Th, ctx->Th, PP * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (sigma_hat) {
    ctx->want_mixed = false;
    RCHK(residual_impl(ctx, ctx->Zs, ctx->opt.singles ? ctx->t1 : nullptr, THC_TERM_ALL));
    RCHK(project_basis(ctx));
    HIPCHK(hipMemcpyAsync(sigma_hat, ctx->sigh, PP * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  }
  return THC_OK;
}


int thc_set_guess_network(thc_ctx* ctx, thc_mlp* net) {
  if (!ctx) return THC_EINVAL;
  if (net && (net->n_in != THC_GUESS_FEATURES || net->w != 256 || net->n_out < 1 || net->n_out > 2 || !net->wb)) {
    ctx->err = "the guess network needs 10 inputs, width 256 and 1 or 2 outputs";
    return THC_EINVAL;
  }
  ctx->guess_net = net;
  return THC_OK;
}

int thc_guess_targets(thc_ctx* ctx, const double* Th0, const double* Tstar, const double* sig0, double* c,
                      double* delta) {
  if (!ctx || !Th0 || !Tstar || !sig0 || !c || !delta) return THC_EINVAL;
  RCHK(need_built(ctx));
  const int64_t P = ctx->P, PP = P * P;
  std::vector<double> T0(PP), Ts(PP), S0(PP), e(P);
  RCHK(d2h(ctx, T0.data(), Th0, PP * sizeof(double)));
  RCHK(d2h(ctx, Ts.data(), Tstar, PP * sizeof(double)));
  RCHK(d2h(ctx, S0.data(), sig0, PP * sizeof(double)));
  RCHK(d2h(ctx, e.data(), ctx->e, P * sizeof(double)));
  // c: Gauss-Newton on s = 1 + c for min || diag(s) T0 diag(s) - T* ||_F, r symmetric:
  //   (J^T r)_k = 2 sum_q r_kq s_q T0_kq,  (J^T J)_kl = 2 d_kl sum_q s_q^2 T0_kq^2 + 2 s_k s_l T0_kl^2
  std::vector<double> sv(P, 1.0), A(PP), b(P);
  for (int it = 0; it < 12; ++it) {
    for (int64_t k = 0; k < P; ++k) {
      double g = 0.0, dsum = 0.0;
      for (int64_t q = 0; q < P; ++q) {
        const double t0 = T0[(size_t)k * P + q];
        const double r = sv[k] * sv[q] * t0 - Ts[(size_t)k * P + q];
        g += r * sv[q] * t0;
        dsum += sv[q] * sv[q] * t0 * t0;
        A[(size_t)k * P + q] = 2.0 * sv[k] * sv[q] * t0 * t0;
      }
      A[(size_t)k * P + k] += 2.0 * dsum;
      b[k] = -2.0 * g;
    }
    if (!spd_solve(P, A, b, 1e-12)) {
      ctx->err = "scaling target: normal matrix not positive definite";
      return THC_ESINGULAR;
    }
    double step = 0.0;
    for (int64_t k = 0; k < P; ++k) {
      sv[k] += b[k];
      step = std::max(step, std::fabs(b[k]));
    }
    if (step < 1e-12) break;
  }
  std::vector<double> ch(P), dh(P);
  for (int64_t k = 0; k < P; ++k) ch[k] = sv[k] - 1.0;
  // delta: normal equations of min sum_PQ (r_PQ - (delta_P + delta_Q) dT_PQ)^2,
  //   r = -sigma0 - (e_P + e_Q) dT:  (diag(rowsum dT^2) + dT o dT) delta = rowsum(r o dT)
  for (int64_t p = 0; p < P; ++p) {
    double rs = 0.0, rhs = 0.0;
    for (int64_t q = 0; q < P; ++q) {
      const double dT = Ts[(size_t)p * P + q] - T0[(size_t)p * P + q];
      const double r = -S0[(size_t)p * P + q] - (e[p] + e[q]) * dT;
      A[(size_t)p * P + q] = dT * dT;
      rs += dT * dT;
      rhs += r * dT;
    }
    A[(size_t)p * P + p] += rs;
    dh[p] = rhs;
  }
  if (!spd_solve(P, A, dh, 1e-10)) {
    ctx->err = "shift target: normal matrix not positive definite";
    return THC_ESINGULAR;
  }
  RCHK(h2d(ctx, c, ch.data(), P * sizeof(double)));
  RCHK(h2d(ctx, delta, dh.data(), P * sizeof(double)));
  return THC_OK;
}

// ------------------------------------------------------------------------------------------
// The learned-guess network.


int thc_mlp_create(int64_t n_in, int64_t width, int64_t n_out, uint64_t seed, void* stream, thc_mlp** out) {
  if (!out || n_in < 1 || width < 1 || n_out < 1 || n_in > 4096 || width > 4096 || n_out > 4096) return THC_EINVAL;
  *out = nullptr;
  thc_mlp* ctx = new (std::nothrow) thc_mlp();
  if (!ctx) return THC_ENOMEM;
  ctx->n_in = n_in;
  ctx->w = width;
  ctx->n_out = n_out;
  ctx->np = n_in * width + width + width * width + width + width * n_out + n_out;
  ctx->stream = (hipStream_t)stream;
  int rc = THC_OK;
  for (float** a : {&ctx->p, &ctx->g, &ctx->m, &ctx->v})
    if (rc == THC_OK) rc = mlp_alloc(ctx, a, (size_t)ctx->np, ctx->allocs);
  for (float** a : {&ctx->mu_in, &ctx->sd_in})
    if (rc == THC_OK) rc = mlp_alloc(ctx, a, (size_t)n_in, ctx->allocs);
  for (float** a : {&ctx->mu_out, &ctx->sd_out})
    if (rc == THC_OK) rc = mlp_alloc(ctx, a, (size_t)n_out, ctx->allocs);
  if (rc == THC_OK) rc = mlp_alloc(ctx, &ctx->loss, 1, ctx->allocs);
  if (rc == THC_OK) rc = mlp_alloc(ctx, &ctx->part, (size_t)MLP_PARTS, ctx->allocs);
  if (rc == THC_OK && mlp_infer_supported(n_in, width, n_out)) {
    rc = mlp_alloc(ctx, &ctx->wb, (size_t)mlp_bf16_weights(n_in), ctx->allocs);
    if (rc == THC_OK) rc = mlp_alloc(ctx, &ctx->bb, (size_t)mlp_bf16_biases(), ctx->allocs);
  }
  if (rc == THC_OK) {
    std::vector<float> zeros((size_t)std::max(n_in, n_out), 0.0f), ones((size_t)std::max(n_in, n_out), 1.0f);
    if (mlp_init(n_in, width, n_out, seed, ctx->p, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->m, 0, ctx->np * sizeof(float), ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->v, 0, ctx->np * sizeof(float), ctx->stream) != hipSuccess)
      rc = THC_EDEVICE;
    if (rc == THC_OK) rc = h2d(ctx, ctx->mu_in, zeros.data(), n_in * sizeof(float));
    if (rc == THC_OK) rc = h2d(ctx, ctx->sd_in, ones.data(), n_in * sizeof(float));
    if (rc == THC_OK) rc = h2d(ctx, ctx->mu_out, zeros.data(), n_out * sizeof(float));
    if (rc == THC_OK) rc = h2d(ctx, ctx->sd_out, ones.data(), n_out * sizeof(float));
  }
  if (rc != THC_OK) {
    for (void* q : ctx->allocs) (void)hipFree(q);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    delete ctx;
    return rc;
  }
  // the allocation-free forward pass's scratch on this device (looked up once per device)
  ctx->scratch_err = mlp_scratch_resolve(&ctx->scratch);
  if (ctx->scratch_err != hipSuccess) (void)hipGetLastError();
  *out = ctx;
  return THC_OK;
}

int thc_mlp_set_norm(thc_mlp* ctx, const float* mu_in, const float* sd_in, const float* mu_out, const float* sd_out) {
  if (!ctx || !mu_in || !sd_in || !mu_out || !sd_out) return THC_EINVAL;
  for (int64_t k = 0; k < ctx->n_in; ++k)
    if (!(sd_in[k] > 0.0f)) { ctx->err = "input scales must be positive"; return THC_EINVAL; }
  for (int64_t k = 0; k < ctx->n_out; ++k)
    if (!(sd_out[k] > 0.0f)) { ctx->err = "output scales must be positive"; return THC_EINVAL; }
  RCHK(h2d(ctx, ctx->mu_in, mu_in, ctx->n_in * sizeof(float)));
  RCHK(h2d(ctx, ctx->sd_in, sd_in, ctx->n_in * sizeof(float)));
  RCHK(h2d(ctx, ctx->mu_out, mu_out, ctx->n_out * sizeof(float)));
  RCHK(h2d(ctx, ctx->sd_out, sd_out, ctx->n_out * sizeof(float)));
  return THC_OK;
}

int thc_mlp_fit_norm(thc_mlp* ctx, const float* X, const float* T, int64_t rows) {
  if (!ctx || !X || !T || rows < 1) return THC_EINVAL;
  HIPCHK(mlp_colstats(rows, ctx->n_in, X, ctx->mu_in, ctx->sd_in, ctx->stream));
  HIPCHK(mlp_colstats(rows, ctx->n_out, T, ctx->mu_out, ctx->sd_out, ctx->stream));
  ctx->packed = false;
  return THC_OK;
}

int thc_mlp_get_norm(thc_mlp* ctx, float* mu_in, float* sd_in, float* mu_out, float* sd_out) {
  if (!ctx || !mu_in || !sd_in || !mu_out || !sd_out) return THC_EINVAL;
  RCHK(d2h(ctx, mu_in, ctx->mu_in, ctx->n_in * sizeof(float)));
  RCHK(d2h(ctx, sd_in, ctx->sd_in, ctx->n_in * sizeof(float)));
  RCHK(d2h(ctx, mu_out, ctx->mu_out, ctx->n_out * sizeof(float)));
  RCHK(d2h(ctx, sd_out, ctx->sd_out, ctx->n_out * sizeof(float)));
  return THC_OK;
}

int thc_mlp_num_params(const thc_mlp* ctx, int64_t* n) {
  if (!ctx || !n) return THC_EINVAL;
  *n = ctx->np;
  return THC_OK;
}

int thc_mlp_get_params(thc_mlp* ctx, float* p) {
  if (!ctx || !p) return THC_EINVAL;
  HIPCHK(hipMemcpyAsync(p, ctx->p, ctx->np * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
  return THC_OK;
}

int thc_mlp_set_params(thc_mlp* ctx, const float* p) {
  if (!ctx || !p) return THC_EINVAL;
  HIPCHK(hipMemcpyAsync(ctx->p, p, ctx->np * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->m, 0, ctx->np * sizeof(float), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->v, 0, ctx->np * sizeof(float), ctx->stream));
  ctx->step = 0;
  ctx->packed = false;
  return THC_OK;
}

int thc_mlp_forward(thc_mlp* ctx, const float* X, int64_t rows, float* Y) {
  if (!ctx || !X || !Y || rows < 0) return THC_EINVAL;
  if (rows == 0) return THC_OK;
  RCHK(mlp_reserve(ctx, rows));
  RCHK(mlp_fwd(ctx, X, rows));
  HIPCHK(mlp_denorm(rows, ctx->n_out, ctx->yn, ctx->mu_out, ctx->sd_out, Y, ctx->stream));
  return THC_OK;
}

int thc_mlp_forward_noalloc(thc_mlp* ctx, const float* X, int64_t rows, float* Y) {
  if (!ctx || !X || !Y || rows < 0) return THC_EINVAL;
  if (rows == 0) return THC_OK;
  if (!ctx->scratch) {
    ctx->err = std::string("thc_mlp_forward_noalloc: the scratch array's device address could not be looked up: ") +
               hipGetErrorString(ctx->scratch_err);
    return THC_EDEVICE;
  }
  const int64_t cap = mlp_scratch_rows(ctx);
  if (rows > cap) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "thc_mlp_forward_noalloc: %lld rows exceed the scratch capacity of %lld rows for this network "
             "(%lld MiB of activations)",
             (long long)rows, (long long)cap, (long long)(MLP_SCRATCH_FLOATS * 4 >> 20));
    ctx->err = buf;
    return THC_EINVAL;
  }
  auto up = [](int64_t n) { return (n + 63) / 64 * 64; };
  const int64_t ni = ctx->n_in, w = ctx->w, no = ctx->n_out;
  float* xn = ctx->scratch;
  float* h1 = xn + up(rows * ni);
  float* h2 = h1 + up(rows * w);
  float* yn = h2 + up(rows * w);
  const float *W1 = ctx->p, *b1 = W1 + ni * w, *W2 = b1 + w, *b2 = W2 + w * w, *W3 = b2 + w, *b3 = W3 + w * no;
  hipStream_t s = ctx->stream;
  HIPCHK(mlp_normalize(rows, ni, X, ctx->mu_in, ctx->sd_in, xn, s));
  HIPCHK(mlp_sgemm(false, false, 4, rows, w, ni, xn, ni, W1, w, h1, w, b1, nullptr, 0, s));
  HIPCHK(mlp_sgemm(false, false, 4, rows, w, w, h1, w, W2, w, h2, w, b2, nullptr, 0, s));
  HIPCHK(mlp_sgemm(false, false, 2, rows, no, w, h2, w, W3, no, yn, no, b3, nullptr, 0, s));
  HIPCHK(mlp_denorm(rows, no, yn, ctx->mu_out, ctx->sd_out, Y, s));
  return THC_OK;
}

int thc_mlp_loss_grad(thc_mlp* ctx, const float* X, const float* T, int64_t rows, float* loss, float* grad) {
  if (!ctx || !X || !T || rows < 1) return THC_EINVAL;
  RCHK(mlp_reserve(ctx, rows));
  RCHK(mlp_bwd(ctx, X, T, rows));
  if (grad) HIPCHK(hipMemcpyAsync(grad, ctx->g, ctx->np * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
  if (loss) {
    RCHK(d2h(ctx, loss, ctx->loss, sizeof(float)));
  }
  return THC_OK;
}

int thc_mlp_train_step(thc_mlp* ctx, const float* X, const float* T, int64_t rows, float lr, float* loss) {
  if (!ctx || !X || !T || rows < 1 || !(lr > 0.0f)) return THC_EINVAL;
  RCHK(mlp_reserve(ctx, rows));
  RCHK(mlp_bwd(ctx, X, T, rows));
  ctx->step += 1;
  HIPCHK(mlp_adam(ctx->np, ctx->p, ctx->g, ctx->m, ctx->v, lr, 0.9f, 0.999f, 1e-8f, ctx->step, ctx->stream));
  ctx->packed = false;
  if (loss) {
    RCHK(d2h(ctx, loss, ctx->loss, sizeof(float)));
  }
  return THC_OK;
}

int thc_mlp_infer(thc_mlp* ctx, const float* X, int64_t rows, float* Y) {
  if (!ctx || !X || !Y || rows < 0) return THC_EINVAL;
  if (!ctx->wb) {
    ctx->err = "BF16 inference needs width 256, n_in <= 16 and n_out <= 16";
    return THC_EINVAL;
  }
  if (!ctx->packed) {
    HIPCHK(mlp_pack_bf16(ctx->n_in, ctx->n_out, ctx->p, ctx->wb, ctx->bb, ctx->stream));
    ctx->packed = true;
  }
  HIPCHK(mlp_infer_bf16(rows, ctx->n_in, ctx->n_out, X, ctx->mu_in, ctx->sd_in, ctx->wb, ctx->bb, ctx->mu_out,
                        ctx->sd_out, Y, ctx->stream));
  return THC_OK;
}

const char* thc_mlp_last_error(const thc_mlp* ctx) { return ctx ? ctx->err.c_str() : "null network"; }

void thc_mlp_destroy(thc_mlp* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (void* q : ctx->acts) (void)hipFree(q);
  for (void* q : ctx->allocs) (void)hipFree(q);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  delete ctx;
}

const char* thc_last_error(const thc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void thc_destroy(thc_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (auto ev : ctx->pool) (void)hipEventDestroy(ev);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  delete ctx;
}

}  // extern "C"
