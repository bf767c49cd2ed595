// Host orchestration of the seeded Chebyshev-filtered subspace iteration and
// the C ABI of libgevp (declared in include/gevp.h).
//
// One solve (the paper's fast iteration, section 2, seeded by the previous
// iteration's eigenvectors):
//   stage    A, B lower triangles -> full Hermitian copies; NaN/Inf scan
//   chol     B = L L^H (blocked, lookahead on a panel stream) with the left
//            solve W = L^{-1} A carried along panel by panel; L^H X0 for a
//            seeded solve, then L^H copied into L's upper triangle
//   reduce   C = W L^{-H} (the lower triangle of the right solve, mirrored)
//   bounds   Lanczos on C (filter interval), on A and B (norm estimates)
//   seed     Y0 = [L^H X0, random], or random for a cold start; a full seed's
//            first projection X0^H A X0 and its eigensolve run on a second
//            stream during the factorisation and reduction
//   loop     CholQR2 -> Rayleigh-Ritz (W = C Y, H = Y^H W, H = Z T Z^H,
//            Y <- Y Z) -> residuals -> controller -> Chebyshev filter
//   final    X = L^{-H} Y(:, 1:kx), original-basis residuals, phase fix,
//            optional seed monitor
// The only device-to-host traffic is a few status words per sweep.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

// Scratch of gevp_backward_noalloc (the only entry point that allocates
// nothing): one array per device, held until the process ends.  In host code
// `scratch` only names the symbol; its device address on each device comes
// from hipGetSymbolAddress, taken once per device by gevp_create.
constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
// device address of `scratch` on the current device `dev` (looked up once)
gevp_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return GEVP_ERR_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GEVP_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return GEVP_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GEVP_OK;
}
}  // namespace

int gevp_log_enabled() {
  static int v = -1;
  if (v < 0) {
    const char* s = getenv("GEVP_LOG");
    v = (s && (s[0] == '1' || s[0] == '2')) ? s[0] - '0' : 0;
  }
  return v;
}

gevp_status ws_reserve(gevp_ctx* c, size_t bytes) {
  c->ws_used = 0;
  if (bytes <= c->ws_bytes) return GEVP_OK;
  if (c->ext) return GEVP_ERR_WORKSPACE;  // the caller's buffer is too small
  if (c->ws) {
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
    GEVP_HIP_TRY(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (hipMalloc((void**)&c->ws, bytes) != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return GEVP_ERR_ALLOC;
  }
  c->ws_bytes = bytes;
  return GEVP_OK;
}

void ext_assign(gevp_ctx* parent, gevp_ctx* child, int slot) {
  if (!parent->ext || !child) return;
  if (child->skw && !child->ext) {
    (void)hipStreamSynchronize(child->stream);
    (void)hipFree(child->skw);
  }
  child->ext = true;
  child->skw = parent->ext_base + parent->ext_bytes - (size_t)(slot + 1) * SKW_BYTES;
  child->skw_bytes = SKW_BYTES;
}

void* ws_take(gevp_ctx* c, size_t bytes) {
  void* p = c->ws + c->ws_used;
  c->ws_used += ws_round(bytes);
  return p;
}

// Event pairs around the filter products (profiling flag 2) and the FP64
// GEMM launches (flag 4); the pools grow on demand and are summed after the
// solve's final synchronisation.
static gevp_status ev_record(gevp_ctx* c, hipEvent_t*& pool, int& cap, int& used) {
  if (used == cap) {
    const int ncap = cap ? 2 * cap : 512;
    hipEvent_t* nv = new hipEvent_t[ncap];
    for (int i = 0; i < cap; ++i) nv[i] = pool[i];
    for (int i = cap; i < ncap; ++i) GEVP_HIP_TRY(hipEventCreate(&nv[i]));
    delete[] pool;
    pool = nv;
    cap = ncap;
  }
  GEVP_HIP_TRY(hipEventRecord(pool[used++], c->stream));
  return GEVP_OK;
}

gevp_status fev_mark(gevp_ctx* c) {
  if (!(c->profiling & 2)) return GEVP_OK;
  return ev_record(c, c->fev, c->fev_cap, c->fev_used);
}

gevp_status gev_begin(gevp_ctx* c) {
  if (!(c->profiling & 4)) return GEVP_OK;
  return ev_record(c, c->gev, c->gev_cap, c->gev_used);
}

gevp_status gev_end(gevp_ctx* c, double flops, const int64_t* shape) {
  if (!(c->profiling & 4)) return GEVP_OK;
  c->gev_flops += flops;
  if (shape && gevp_log_enabled() >= 2) {
    for (int i = 0; i < 6; ++i) c->gev_shape.push_back((double)shape[i]);
    c->gev_shape.push_back(flops);
  }
  return ev_record(c, c->gev, c->gev_cap, c->gev_used);
}

namespace {

struct Opts {
  int precision, nex, deg_init, deg_max, maxit, lanczos;
  unsigned long long seed;
  int skip_final;
  int seed_monitor;
  int filter, nq;
  int lock_mode;
  int sweep_reduction;  // log10 of a low-precision sweep's largest aimed reduction (0: default)
  int deg_reach;        // degree cap of a sweep that can finish the solve (>= deg_max)
};

Opts resolve(const gevp_opts* o, int64_t nev) {
  Opts r;
  r.precision = o ? o->precision : 0;
  r.nex = o ? o->nex : 0;
  if (r.nex <= 0) {
    int64_t x = (int64_t)std::ceil(0.15 * (double)nev);
    if (x < 16) x = 16;
    r.nex = (int)((x + 15) / 16 * 16);
  }
  r.deg_init = (o && o->deg_init > 0) ? o->deg_init : 20;
  r.deg_max = (o && o->deg_max > 0) ? o->deg_max : 36;
  if (r.deg_max > 200) r.deg_max = 200;
  if (r.deg_init > r.deg_max) r.deg_init = r.deg_max;
  r.deg_reach = std::min(200, r.deg_max + r.deg_max / 3);
  r.maxit = (o && o->maxit > 0) ? o->maxit : 40;
  r.lanczos = (o && o->lanczos_steps > 0) ? o->lanczos_steps : 24;
  r.seed = o ? o->seed : 0ull;
  r.skip_final = o ? o->skip_final_residual : 0;
  r.seed_monitor = o ? o->seed_monitor : 0;
  r.filter = o ? o->filter : 0;
  r.nq = (o && o->contour_points > 0) ? o->contour_points : 8;
  r.lock_mode = o ? o->lock_mode : 0;
  r.sweep_reduction = (o && o->sweep_reduction > 0 && o->sweep_reduction < 16) ? o->sweep_reduction : 0;
  return r;
}

int64_t block_of(const Opts& o, int64_t n, int64_t nev) {
  int64_t nb = nev + o.nex;
  return nb > n ? n : nb;
}

// Device workspace of one gevp_solve (the pieces carved below, in order).
size_t solve_ws_bytes(const Opts& o, int64_t n, int64_t nb, bool contour, bool c32, bool lp,
                      bool bf16) {
  const size_t nn = (size_t)n * n;
  const int lz = o.lanczos;
  size_t need = 0;
  need += 4 * ws_round(sizeof(zd) * nn);                 // Af, Bf, L, C
  need += ws_round(sizeof(zd) * n * 64);                 // Dinv
  need += 4 * ws_round(sizeof(zd) * n * nb);             // P0, P1, W, T
  need += 3 * ws_round(sizeof(zd) * nb * nb);            // H, Z, G
  need += ws_round(sizeof(zd) * nb * 64);                // DinvG
  need += heev_work_bytes(nb);
  need += 2 * lanczos_work_bytes(n, lz);                 // main and second stream
  need += 3 * ws_round(sizeof(double) * 8);              // bounds C, A, B
  need += 4 * ws_round(sizeof(double) * nb);             // theta, resid, final residuals, merge order
  need += ws_round(sizeof(int) * nb);                    // perm
  need += ws_round(sizeof(double) * 3 * 256);            // coefs
  need += ws_round(sizeof(int) * 300) + ws_round(sizeof(double) * 16);  // status
  need += ws_round(sizeof(int) * 8) + ws_round(sizeof(double) * 8);     // flags, shift
  need += ws_round(sizeof(double) * 4);                  // norms
  need += ws_round(sizeof(double) * (3 * nb + 8));       // seed monitor
  if (o.seed_monitor)  // the seed in the reduced basis and its projection residual norms
    need += ws_round(sizeof(zd) * n * nb) + ws_round(sizeof(double) * nb);
  if (contour)  // nq factorisations
    need += c32 ? contour32_work_bytes(n, nb, o.nq) : contour_work_bytes(n, nb, o.nq);
  const size_t lp_elem = 8;                              // complex64
  if (lp) {
    need += bf16 ? ws_round(bf16_planes_bytes(n)) : ws_round(lp_elem * nn);  // low-precision C
    if (bf16) need += bf16_filter_work_bytes(n, nb);     // iterate planes, split-K partials
    need += 3 * ws_round(lp_elem * n * nb);              // G0, G1, R (low precision)
    need += ws_round(sizeof(double) * nb);               // rho0
    need += ws_round(sizeof(double) * 4 * nb * (o.deg_reach + 2));  // per-column coefficients
  }
  return need;
}

// Worst case over seeds: the contour filter's factorisations when it is
// selected, the low-precision Chebyshev buffers for a mixed precision (a
// solve that cannot place a contour takes the Chebyshev filter).
size_t solve_ws_bytes_max(const Opts& o, int64_t n, int64_t nev) {
  const int64_t nb = block_of(o, n, nev);
  const bool mixed = o.precision != GEVP_FP64;
  const bool contour = o.filter == GEVP_FILTER_CONTOUR && nb > nev && n <= 65535;
  size_t b = solve_ws_bytes(o, n, nb, false, false, mixed, o.precision == GEVP_BF16X3);
  if (contour)
    b = std::max(b, solve_ws_bytes(o, n, nb, true, mixed, false, false));
  return b;
}

struct Timer {
  gevp_ctx* c;
  hipEvent_t ev[2];
  bool on;
  Timer(gevp_ctx* ctx) : c(ctx), on((ctx->profiling & 1) != 0) {
    if (on) {
      (void)hipEventCreate(&ev[0]);
      (void)hipEventCreate(&ev[1]);
    }
  }
  ~Timer() {
    if (on) {
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
    }
  }
  void start() {
    if (on) (void)hipEventRecord(ev[0], c->stream);
  }
  void stop(gevp_info* info, int stage) {
    if (!on) return;
    (void)hipEventRecord(ev[1], c->stream);
    (void)hipEventSynchronize(ev[1]);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (info) info->ms[stage] += ms;
  }
};

// Orthonormalise the m columns of P (n x m) by CholQR2 with column scaling;
// a failed Cholesky of the Gram matrix falls back to a shifted first pass.
struct QrWork {
  zd* G;
  zd* Dg;
  int* flag;
  double* shift;
};

// try_skip: the block may already be orthonormal (a seed from the previous
// step with an unchanged overlap): if the first Gram matrix is the identity
// to 1e-11, no factorisation is needed.  Such a seed deviates from I by the
// rounding of L^H X0 and of the previous solve (1.5e-13 .. 5.3e-13 measured
// at n = 8192, where a 5e-13 bound rejected half the steps); its Ritz pairs
// only start the iteration, and the next sweep orthonormalises in full.
gevp_status cholqr2(gevp_ctx* c, int64_t n, int64_t m, zd* P, int64_t ldp, QrWork& w,
                    int* fallbacks, bool try_skip = false, bool* skipped = nullptr) {
  if (skipped) *skipped = false;
  for (int pass = 0; pass < 2; ++pass) {
    GEVP_TRY(launch_colnorm_scale(c, n, m, P, ldp));
    // the Gram matrix's lower triangle only: the factorisation and the check
    // below read nothing else
    GEVP_TRY(launch_zgemm(c, 1, 0, m, m, n, 1.0, P, ldp, P, ldp, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, w.G, m, nullptr, 1));
    // An orthonormal seed needs no pass at all, and a first pass that already
    // left the block orthonormal to 5e-13 needs no second one: the Gram
    // matrix is formed either way, and the check replaces the host read of
    // the Cholesky's status.
    if ((pass == 0 && try_skip) || pass == 1) {
      double dev = 1.0;
      // partial maxima in Dg, whose inverse blocks the last solve has consumed
      GEVP_TRY(launch_max_offident(c, m, w.G, m, w.shift + 1, reinterpret_cast<double*>(w.Dg)));
      GEVP_HIP_TRY(hipMemcpyAsync(&dev, w.shift + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
      if (gevp_log_enabled())
        fprintf(stderr, "[gevp] cholqr pass %d m %lld: max |G - I| %.3e\n", pass, (long long)m, dev);
      if (dev <= (pass == 0 ? 1e-11 : 5e-13)) {
        if (skipped && pass == 0) *skipped = true;
        return GEVP_OK;
      }
    }
    const int big = 0x7fffffff;
    GEVP_HIP_TRY(hipMemcpyAsync(w.flag, &big, sizeof(int), hipMemcpyHostToDevice, c->stream));
    GEVP_TRY(chol_lower(c, m, w.G, m, w.Dg, m, w.flag));
    int f = big;
    GEVP_HIP_TRY(hipMemcpyAsync(&f, w.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
    if (f != big) {
      // shifted CholQR (Fukaya et al.): G + s I with s = 11 (n m + m (m+1)) u ||G||,
      // ||G|| <= trace(G) = m after column scaling; then two more plain passes
      ++*fallbacks;
      const double u = 1.1102230246251565e-16;
      const double s = 11.0 * ((double)n * m + (double)m * (m + 1)) * u * (double)m;
      GEVP_TRY(launch_zgemm(c, 1, 0, m, m, n, 1.0, P, ldp, P, ldp, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, w.G, m, nullptr, 1));
      GEVP_HIP_TRY(hipMemcpyAsync(w.shift, &s, sizeof(double), hipMemcpyHostToDevice, c->stream));
      GEVP_TRY(launch_add_diag(c, m, w.G, m, w.shift));
      GEVP_HIP_TRY(hipMemcpyAsync(w.flag, &big, sizeof(int), hipMemcpyHostToDevice, c->stream));
      GEVP_TRY(chol_lower(c, m, w.G, m, w.Dg, m, w.flag));
      GEVP_TRY(trsm_right_lower_c(c, m, n, w.G, m, w.Dg, m, P, ldp));
      pass = -1;  // two plain passes follow
      if (*fallbacks > 8) return GEVP_ERR_NOCONV;
      continue;
    }
    GEVP_TRY(trsm_right_lower_c(c, m, n, w.G, m, w.Dg, m, P, ldp));
  }
  return GEVP_OK;
}

gevp_status fev_collect(gevp_ctx* c, gevp_info* info) {
  if (!(c->profiling & 2)) return GEVP_OK;
  double tot = 0.0;
  for (int i = 0; i + 1 < c->fev_used; i += 2) {
    float ms = 0.f;
    GEVP_HIP_TRY(hipEventElapsedTime(&ms, c->fev[i], c->fev[i + 1]));
    tot += ms;
  }
  info->filter_kernel_ms += tot;
  info->filter_launches += c->fev_used / 2;
  c->fev_used = 0;
  return GEVP_OK;
}

// FP64 GEMM launches of a context (and of the streams it forks): summed into
// info once their work has completed
gevp_status gev_collect(gevp_ctx* c, gevp_info* info) {
  if (!c || !(c->profiling & 4)) return GEVP_OK;
  double tot = 0.0;
  for (int i = 0; i + 1 < c->gev_used; i += 2) {
    float ms = 0.f;
    GEVP_HIP_TRY(hipEventElapsedTime(&ms, c->gev[i], c->gev[i + 1]));
    tot += ms;
    const size_t r = (size_t)(i / 2) * 7;
    if (r + 7 <= c->gev_shape.size()) {
      const double* g = c->gev_shape.data() + r;
      static const char* form[4] = {"NN", "NC", "CN", "CC"};
      fprintf(stderr, "[gevp] gemm stream %p %s m %lld n %lld k %lld split %lld wg %lld %.4f ms %.1f TFLOP/s\n",
              (void*)c->stream, form[(int)g[0] & 3], (long long)g[1], (long long)g[2], (long long)g[3],
              (long long)g[4], (long long)g[5], ms, ms > 0 ? g[6] / (ms * 1e9) : 0.0);
    }
  }
  c->gev_shape.clear();
  info->gemm_kernel_ms += tot;
  info->gemm_launches += c->gev_used / 2;
  info->gemm_flops += c->gev_flops;
  c->gev_used = 0;
  c->gev_flops = 0.0;
  return GEVP_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* gevp_status_string(gevp_status s) {
  switch (s) {
    case GEVP_OK: return "ok";
    case GEVP_ERR_INVALID: return "invalid argument";
    case GEVP_ERR_NOT_HPD: return "B is not Hermitian positive definite";
    case GEVP_ERR_NOCONV: return "not converged";
    case GEVP_ERR_HIP: return "HIP runtime error";
    case GEVP_ERR_NONFINITE: return "NaN or Inf in the input";
    case GEVP_ERR_ALLOC: return "workspace allocation failed";
    case GEVP_ERR_SINGULAR: return "zero or non-finite pivot in a shifted factorisation";
    case GEVP_ERR_WORKSPACE: return "caller-provided workspace too small";
  }
  return "unknown status";
}

gevp_status gevp_create(gevp_handle* h, int device) {
  if (!h) return GEVP_ERR_INVALID;
  *h = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return GEVP_ERR_HIP;
  }
  // set-up of the no-allocation entry point: the device address of this
  // device's scratch array, with the device current
  void* sp = nullptr;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = device;
  const bool ok = hipSetDevice(device) == hipSuccess && scratch_address(device, &sp) == GEVP_OK;
  (void)hipSetDevice(prev);
  if (!ok) {
    (void)hipGetLastError();
    return GEVP_ERR_HIP;
  }
  gevp_ctx* c = new gevp_ctx();
  c->device = device;
  *h = c;
  return GEVP_OK;
}

gevp_status gevp_set_stream(gevp_handle h, void* s) {
  if (!h) return GEVP_ERR_INVALID;
  h->stream = (hipStream_t)s;
  return GEVP_OK;
}

gevp_status gevp_set_profiling(gevp_handle h, int on) {
  if (!h) return GEVP_ERR_INVALID;
  h->profiling = on;
  return GEVP_OK;
}

void gevp_destroy(gevp_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  for (gevp_ctx* w : h->workers) gevp_destroy(w);
  h->workers.clear();
  for (gevp_ctx* w : h->qctx) gevp_destroy(w);
  h->qctx.clear();
  if (h->aux) gevp_destroy(h->aux);
  h->aux = nullptr;
  if (h->panel) gevp_destroy(h->panel);
  h->panel = nullptr;
  for (hipEvent_t& e : h->pev)
    if (e) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(h->stream);
  for (gevp_ctx::GraphEntry& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->owns_stream) (void)hipStreamDestroy(h->stream);
  if (h->ws && !h->ext) (void)hipFree(h->ws);
  if (h->skw && !h->ext) (void)hipFree(h->skw);
  for (int i = 0; i < h->fev_cap; ++i) (void)hipEventDestroy(h->fev[i]);
  delete[] h->fev;
  for (int i = 0; i < h->gev_cap; ++i) (void)hipEventDestroy(h->gev[i]);
  delete[] h->gev;
  delete h;
}

int64_t gevp_block_size(const gevp_opts* opts, int64_t n, int64_t nev) {
  if (n < 1 || nev < 1 || nev > n) return 0;
  return block_of(resolve(opts, nev), n, nev);
}

gevp_status gevp_workspace_size(gevp_handle h, const gevp_opts* opts, int64_t n, int64_t nev,
                                size_t* bytes) {
  (void)h;  // the size depends on the arguments only
  if (!bytes || n < 1 || nev < 1 || nev > n) return GEVP_ERR_INVALID;
  const Opts o = resolve(opts, nev);
  *bytes = solve_ws_bytes_max(o, n, nev) + (size_t)EXT_SLOTS * SKW_BYTES;
  return GEVP_OK;
}

namespace {
int batch_stream_count(const gevp_opts* opts, int count) {
  int streams = (opts && opts->batch_streams > 0) ? opts->batch_streams : 8;
  if (streams > 16) streams = 16;
  if (streams > count) streams = count;
  return streams;
}
// per-worker share of a caller-owned workspace in gevp_solve_batched: the
// worker's solve workspace followed by its split-K buffer
size_t worker_share(gevp_ctx* h, int streams) {
  return (h->ext_bytes / (size_t)streams) & ~size_t(255);
}
}  // namespace

gevp_status gevp_workspace_size_batched(gevp_handle h, const gevp_opts* opts, int count,
                                        const int64_t* n, const int64_t* nev, size_t* bytes) {
  (void)h;
  if (!bytes || count < 1 || !n || !nev) return GEVP_ERR_INVALID;
  size_t per = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || nev[i] < 1 || nev[i] > n[i]) return GEVP_ERR_INVALID;
    per = std::max(per, solve_ws_bytes_max(resolve(opts, nev[i]), n[i], nev[i]));
  }
  per = ws_round(per + SKW_BYTES);
  const size_t total = per * (size_t)batch_stream_count(opts, count);
  *bytes = std::max(total, (size_t)EXT_SLOTS * SKW_BYTES + 256);
  return GEVP_OK;
}

gevp_status gevp_set_workspace(gevp_handle h, void* dev_ptr, size_t bytes) {
  if (!h) return GEVP_ERR_INVALID;
  if (dev_ptr && (((uintptr_t)dev_ptr & 255) != 0 || bytes < (size_t)EXT_SLOTS * SKW_BYTES + 256))
    return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  GEVP_HIP_TRY(hipStreamSynchronize(h->stream));
  std::vector<gevp_ctx*> subs = {h->aux, h->panel};
  for (gevp_ctx* q : h->qctx) subs.push_back(q);
  for (gevp_ctx* w : h->workers) subs.push_back(w);
  // release what the library allocated itself; forget borrowed memory
  auto drop = [](gevp_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (!c->ext) {
      if (c->ws) (void)hipFree(c->ws);
      if (c->skw) (void)hipFree(c->skw);
    }
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->ws_used = 0;
    c->skw = nullptr;
    c->skw_bytes = 0;
    c->ext = false;
  };
  drop(h);
  for (gevp_ctx* c : subs) drop(c);
  h->ext_base = nullptr;
  h->ext_bytes = 0;
  if (!dev_ptr) return GEVP_OK;  // back to library-managed memory
  h->ext = true;
  h->ext_base = (char*)dev_ptr;
  h->ext_bytes = bytes;
  h->ws = h->ext_base;
  h->ws_bytes = bytes - (size_t)EXT_SLOTS * SKW_BYTES;
  h->skw = h->ext_base + bytes - SKW_BYTES;  // slot SLOT_MAIN
  h->skw_bytes = SKW_BYTES;
  ext_assign(h, h->aux, SLOT_AUX);
  ext_assign(h, h->panel, SLOT_PANEL);
  for (size_t q = 0; q < h->qctx.size(); ++q) ext_assign(h, h->qctx[q], SLOT_QUAD0 + (int)q);
  return GEVP_OK;
}

namespace {
// the handle's second stream (non-blocking, default priority), created once
gevp_status aux_ctx(gevp_ctx* c, gevp_ctx** out) {
  if (!c->aux) {
    gevp_ctx* w = new gevp_ctx();
    w->device = c->device;
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      return GEVP_ERR_HIP;
    }
    w->owns_stream = true;
    c->aux = w;
    ext_assign(c, w, SLOT_AUX);
  }
  *out = c->aux;
  return GEVP_OK;
}

// Fork/join events of the second stream.  Every exit from the solve, early
// error returns included, waits for the second stream's work first: it reads
// the caller's X0 and writes workspace the next call reuses.
struct EventPair {
  hipEvent_t fork = nullptr, mid = nullptr, join = nullptr;
  hipEvent_t reduced = nullptr, bounds = nullptr;  // C formed; its Lanczos bound done
  hipStream_t second = nullptr;  // set once work is queued on the second stream
  ~EventPair() {
    if (second) (void)hipStreamSynchronize(second);
    for (hipEvent_t e : {fork, mid, join, reduced, bounds})
      if (e) (void)hipEventDestroy(e);
  }
};
}  // namespace

gevp_status gevp_solve(gevp_handle h, const gevp_opts* opts, int64_t n, const void* A_,
                       int64_t lda, const void* B_, int64_t ldb, const void* X0_, int64_t ldx0,
                       int64_t k0, int64_t nev, double tol, int64_t kx, double* lambda, void* X_,
                       int64_t ldx, double* resid_out, gevp_info* info) {
  gevp_info dummy;
  if (!info) info = &dummy;
  std::memset(info, 0, sizeof(*info));
  info->seed_sin_rms = info->seed_dev_mean = info->seed_dev_max = info->seed_dev_std = -1.0;
  auto bad = [&](int arg) {
    info->lapack_info = -arg;
    return GEVP_ERR_INVALID;
  };
  if (!h) return bad(1);
  if (n < 1) return bad(3);
  if (!A_ || lda < n) return bad(5);
  if (!B_ || ldb < n) return bad(7);
  if (nev < 1 || nev > n) return bad(11);
  if (!(tol > 0.0)) return bad(12);
  const Opts o = resolve(opts, nev);
  if (o.precision != GEVP_FP64 && o.precision != GEVP_FP32 && o.precision != GEVP_BF16X3)
    return bad(2);
  if (o.filter != GEVP_FILTER_CHEBYSHEV && o.filter != GEVP_FILTER_CONTOUR) return bad(2);
  if (o.nq < 1 || o.nq > 256) return bad(2);
  const bool mixed = (o.precision != GEVP_FP64);
  const bool bf16 = (o.precision == GEVP_BF16X3);
  const int64_t nb = block_of(o, n, nev);
  if (kx < nev || kx > nb) return bad(13);
  if (X0_ && k0 > 0 && (ldx0 < n || k0 > nb)) return bad(10);
  if (k0 < 0) return bad(10);
  if (!lambda) return bad(14);
  if (!X_ || ldx < n) return bad(16);
  if (nb > 2048) return bad(11);  // Rayleigh-Ritz eigensolver limit
  const bool seeded = (X0_ != nullptr && k0 > 0);
  // the contour filter places its circle from the seed's Ritz values, which
  // needs the first unwanted one (column nev) to come from the seed
  const bool contour =
      o.filter == GEVP_FILTER_CONTOUR && seeded && k0 > nev && nb > nev && n <= 65535;
  const bool lp = mixed && !contour;  // low-precision Chebyshev filter in use
  const bool c32 = contour && mixed;  // contour filter in FP32, residual-correction form
  GEVP_HIP_TRY(hipSetDevice(h->device));
  gevp_ctx* c = h;
  c->fev_used = 0;
  c->gev_used = 0;
  c->gev_flops = 0.0;
  info->block = (int)nb;

  const zd* A = (const zd*)A_;
  const zd* B = (const zd*)B_;
  const zd* X0 = (const zd*)X0_;
  zd* X = (zd*)X_;

  // ---------------- workspace
  const size_t nn = (size_t)n * n;
  const int lz = o.lanczos;
  const size_t lp_elem = 8;                              // complex64
  const size_t need = solve_ws_bytes(o, n, nb, contour, c32, lp, bf16);
  GEVP_TRY(ws_reserve(c, need));
  zd* Af = (zd*)ws_take(c, sizeof(zd) * nn);
  zd* Bf = (zd*)ws_take(c, sizeof(zd) * nn);
  zd* L = (zd*)ws_take(c, sizeof(zd) * nn);
  zd* C = (zd*)ws_take(c, sizeof(zd) * nn);
  zd* Dinv = (zd*)ws_take(c, sizeof(zd) * n * 64);
  zd* P0 = (zd*)ws_take(c, sizeof(zd) * n * nb);
  zd* P1 = (zd*)ws_take(c, sizeof(zd) * n * nb);
  // W and T adjacent: the final residual stacks [A X; B X] over both
  zd* const WT = (zd*)ws_take(c, sizeof(zd) * 2 * n * nb);
  zd* W = WT;
  zd* T = WT + n * nb;
  zd* Hs = (zd*)ws_take(c, sizeof(zd) * nb * nb);
  zd* Zs = (zd*)ws_take(c, sizeof(zd) * nb * nb);
  zd* Gs = (zd*)ws_take(c, sizeof(zd) * nb * nb);
  zd* DinvG = (zd*)ws_take(c, sizeof(zd) * nb * 64);
  void* heevw = ws_take(c, heev_work_bytes(nb));
  void* lanw = ws_take(c, lanczos_work_bytes(n, lz));
  void* lanw2 = ws_take(c, lanczos_work_bytes(n, lz));
  double* bC = (double*)ws_take(c, sizeof(double) * 8);
  double* bA = (double*)ws_take(c, sizeof(double) * 8);
  double* bB = (double*)ws_take(c, sizeof(double) * 8);
  double* theta = (double*)ws_take(c, sizeof(double) * nb);
  double* rres = (double*)ws_take(c, sizeof(double) * nb);
  double* fres = (double*)ws_take(c, sizeof(double) * nb);
  int* order = (int*)ws_take(c, sizeof(double) * nb);  // merge order of the locked sweep
  int* perm = (int*)ws_take(c, sizeof(int) * nb);
  double* coefs = (double*)ws_take(c, sizeof(double) * 3 * 256);
  int* st_i = (int*)ws_take(c, sizeof(int) * 300);
  double* st_d = (double*)ws_take(c, sizeof(double) * 16);
  int* flags = (int*)ws_take(c, sizeof(int) * 8);
  double* shift = (double*)ws_take(c, sizeof(double) * 8);
  double* norms = (double*)ws_take(c, sizeof(double) * 4);
  double* mon = (double*)ws_take(c, sizeof(double) * (3 * nb + 8));  // per-column stats, then 6 results
  const int64_t km = std::min<int64_t>(nev, k0);
  const bool monitor = seeded && o.seed_monitor && km > 0;
  zd* Y0s = o.seed_monitor ? (zd*)ws_take(c, sizeof(zd) * n * nb) : nullptr;
  double* rmon = o.seed_monitor ? (double*)ws_take(c, sizeof(double) * nb) : nullptr;
  void* cw = contour ? ws_take(c, c32 ? contour32_work_bytes(n, nb, o.nq)
                                       : contour_work_bytes(n, nb, o.nq))
                     : nullptr;
  void* Clp = nullptr;
  void* bfw = nullptr;  // split-BF16 filter workspace
  void* G0 = nullptr;
  void* G1 = nullptr;
  void* Rlp = nullptr;
  double* rho0 = nullptr;
  double* coef2 = nullptr;
  if (lp) {
    Clp = ws_take(c, bf16 ? bf16_planes_bytes(n) : lp_elem * nn);
    if (bf16) bfw = ws_take(c, bf16_filter_work_bytes(n, nb));
    G0 = ws_take(c, lp_elem * n * nb);
    G1 = ws_take(c, lp_elem * n * nb);
    Rlp = ws_take(c, lp_elem * n * nb);
    rho0 = (double*)ws_take(c, sizeof(double) * nb);
    coef2 = (double*)ws_take(c, sizeof(double) * 4 * nb * (o.deg_reach + 2));
  }

  Timer tm(c);
  // flags[0]: nonfinite input, flags[1]: Cholesky pivot of B, flags[2]: QR flag
  int init_flags[4] = {0, 0x7fffffff, 0x7fffffff, 0};
  GEVP_HIP_TRY(hipMemcpyAsync(flags, init_flags, sizeof(init_flags), hipMemcpyHostToDevice, c->stream));

  // ---------------- stage
  tm.start();
  GEVP_TRY(launch_mirror_lower(c, n, A, lda, Af, n, flags));
  GEVP_TRY(launch_mirror_lower(c, n, B, ldb, Bf, n, flags));
  if (seeded) GEVP_TRY(launch_check_finite(c, n, k0, X0, ldx0, flags));
  tm.stop(info, GEVP_STAGE_STAGE);

  // A full seed block X0 is B-orthonormal when the overlap matrix has not
  // changed; then its Rayleigh-Ritz projection needs no reduced matrix:
  // (L^H X0)^H C (L^H X0) = X0^H A X0.  The projection, its eigensolve and
  // the norm estimates of A and B run on a second stream: the estimates
  // during the first half of the Cholesky factorisation, the projection
  // from its middle on (the second half leaves most compute units idle)
  // into the reduction.  The projection is used if the
  // orthonormality test of L^H X0 at the first iteration passes (the usual
  // path runs otherwise).  The second stream writes only T, Hs, Zs, theta,
  // norms, its Lanczos workspace and the eigensolver workspace, none of
  // which the main stream touches before the join.
  const bool full_seed = seeded && k0 >= nb;
  const bool spec = full_seed && c->inner_streams;
  const int lzn = lz > 12 ? 12 : lz;  // norm estimates need fewer steps than the filter bound
  const double frac = std::min(1.0, (double)nb / (double)n);
  EventPair evs;
  gevp_ctx* ax = nullptr;
  if (spec) {
    GEVP_TRY(aux_ctx(c, &ax));
    ax->profiling = c->profiling & 4;
    ax->gev_used = 0;
    ax->gev_flops = 0.0;
    GEVP_HIP_TRY(hipEventCreateWithFlags(&evs.fork, hipEventDisableTiming));
    GEVP_HIP_TRY(hipEventCreateWithFlags(&evs.mid, hipEventDisableTiming));
    GEVP_HIP_TRY(hipEventCreateWithFlags(&evs.join, hipEventDisableTiming));
    GEVP_HIP_TRY(hipEventCreateWithFlags(&evs.reduced, hipEventDisableTiming));
    GEVP_HIP_TRY(hipEventCreateWithFlags(&evs.bounds, hipEventDisableTiming));
    // norm estimates (bandwidth-bound) overlap the first, GEMM-bound half of
    // the factorisation
    GEVP_HIP_TRY(hipEventRecord(evs.fork, c->stream));
    GEVP_HIP_TRY(hipStreamWaitEvent(ax->stream, evs.fork, 0));
    evs.second = ax->stream;
    auto norms2 = [&]() -> gevp_status {
      GEVP_TRY(lanczos_bounds(ax, n, Af, n, lzn, o.seed ^ 0xA11CEull, frac, bA, lanw2));
      GEVP_TRY(lanczos_bounds(ax, n, Bf, n, lzn, o.seed ^ 0xB0Bull, frac, bB, lanw2));
      GEVP_TRY(launch_copy_real(ax, 1, bA + 5, norms));
      return launch_copy_real(ax, 1, bB + 5, norms + 1);
    };
    GEVP_TRY(norms2());
  }

  // ---------------- Cholesky of B
  // (with the first half of the reduction, W = L^{-1} A, carried along the
  // factorisation: C starts as a copy of A)
  tm.start();
  GEVP_TRY(launch_copy2d(c, n, n, Bf, n, L, n));
  GEVP_TRY(launch_copy2d(c, n, n, Af, n, C, n));
  GEVP_TRY(chol_lower(c, n, L, n, Dinv, n, flags + 1, spec ? evs.mid : nullptr, C, n, n));
  tm.stop(info, GEVP_STAGE_CHOL);
  if (spec) {  // second stream, from the Cholesky's midpoint on
    GEVP_HIP_TRY(hipStreamWaitEvent(ax->stream, evs.mid, 0));
    auto second = [&]() -> gevp_status {
      GEVP_TRY(launch_zgemm(ax, 0, 0, n, nb, n, 1.0, Af, n, X0, ldx0, 0.0, nullptr, 0, 0.0, nullptr,
                            0, nullptr, T, n));
      GEVP_TRY(launch_zgemm(ax, 1, 0, nb, nb, n, 1.0, X0, ldx0, T, n, 0.0, nullptr, 0, 0.0, nullptr,
                            0, nullptr, Hs, nb, nullptr, 1));
      GEVP_TRY(launch_mirror_lower(ax, nb, Hs, nb, Hs, nb, nullptr));
      return heev_small(ax, nb, Hs, nb, theta, Zs, nb, heevw);
    };
    const gevp_status sst = second();
    GEVP_HIP_TRY(hipEventRecord(evs.join, ax->stream));
    GEVP_TRY(sst);
  }

  int hf[2];
  GEVP_HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, c->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
  if (hf[0]) return GEVP_ERR_NONFINITE;
  if (hf[1] != 0x7fffffff) {
    info->lapack_info = n + hf[1];
    return GEVP_ERR_NOT_HPD;
  }

  // from here on the upper triangle of L holds L^H, so the products and
  // solves with L^H multiply blocks as stored (the faster operand form of the
  // GEMM)
  GEVP_TRY(launch_mirror_lower(c, n, L, n, L, n, flags + 3));
  // C-space seed y = L^H x: the upper triangle of L as stored (the product
  // skips the K range below each row block's diagonal)
  if (seeded)
    GEVP_TRY(launch_zgemm(c, 0, 0, n, k0, n, 1.0, L, n, X0, ldx0, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, P0, n, nullptr, 0, 1));
  if (monitor) GEVP_TRY(launch_copy2d(c, n, km, P0, n, Y0s, n));  // the seed y0 = L^H x0, kept

  // ---------------- reduction to standard form
  tm.start();
  // C = W L^{-H} (W = L^{-1} A, formed with the factorisation) is Hermitian:
  // only its lower triangle is formed, then mirrored
  GEVP_TRY(trsm_right_lower_c_lowerpart(c, n, L, n, Dinv, n, C, n, 1));
  GEVP_TRY(launch_mirror_lower(c, n, C, n, C, n, flags + 3));
  if (lp && bf16) GEVP_TRY(launch_split_rows_bf16(c, n, C, n, Clp));
  if (lp && !bf16) GEVP_TRY(launch_to_c32(c, n, n, C, n, Clp, n));
  tm.stop(info, GEVP_STAGE_REDUCE);

  // ---------------- bounds
  tm.start();
  if (spec) {
    // the bound of C (bandwidth-bound) goes to the second stream, after its
    // seed eigensolve, and overlaps the first rotation and C P (GEMM-bound);
    // the main stream waits for it just before the first controller call
    GEVP_HIP_TRY(hipEventRecord(evs.reduced, c->stream));
    GEVP_HIP_TRY(hipStreamWaitEvent(ax->stream, evs.reduced, 0));
    GEVP_TRY(lanczos_bounds(ax, n, C, n, lz, o.seed ^ 0xC0FFEEull, frac, bC, lanw2));
    GEVP_HIP_TRY(hipEventRecord(evs.bounds, ax->stream));
  } else {
    GEVP_TRY(lanczos_bounds(c, n, C, n, lz, o.seed ^ 0xC0FFEEull, frac, bC, lanw));
  }
  if (!spec) {
    GEVP_TRY(lanczos_bounds(c, n, Af, n, lzn, o.seed ^ 0xA11CEull, frac, bA, lanw));
    GEVP_TRY(lanczos_bounds(c, n, Bf, n, lzn, o.seed ^ 0xB0Bull, frac, bB, lanw));
    GEVP_TRY(launch_copy_real(c, 1, bA + 5, norms));
    GEVP_TRY(launch_copy_real(c, 1, bB + 5, norms + 1));
  }
  tm.stop(info, GEVP_STAGE_BOUNDS);

  // ---------------- initial block
  const int64_t kseed = seeded ? k0 : 0;
  GEVP_TRY(launch_randn(c, n, nb - kseed, P0 + kseed * n, n, kseed, o.seed));

  QrWork qw{Gs, DinvG, flags + 2, shift};
  int fallbacks = 0;
  // rounding floor of the filter products: FP32 products with FP32
  // accumulation over n terms, or split-BF16 products (about 2^-16 each)
  const double u_target =
      o.sweep_reduction > 0 ? std::pow(10.0, -o.sweep_reduction) : (bf16 ? 1e-4 : 1e-6);
  // the degree model is a first-order estimate: aiming a few times below tol
  // lets the columns it slightly misjudges converge in the same sweep instead
  // of costing another orthonormalisation and Rayleigh-Ritz round
  const double margin = 4.0;
  // a sweep whose every wanted column needs at most 5 / u_target more may aim
  // for the tolerance at once, up to deg_reach: measured on the n = 8192
  // sequence, steps whose seed residuals need <= 5e4 (split-BF16) then finish
  // after one filtered sweep instead of two; an explicit sweep_reduction
  // keeps its fixed cap
  const double u_reach = o.sweep_reduction > 0 ? 0.0 : u_target / 5.0;
  CtlParams cp{(int)nb, (int)nev, o.deg_max, o.deg_init, 0, u_target, margin, u_reach, o.deg_reach};
  std::vector<int> hst(4 + 260);
  std::vector<double> hsd(16);
  int it = 0;
  bool converged = false;
  bool need_filter_first = !seeded && nb < n;
  gevp_status st = GEVP_OK;

  auto run_filter = [&](int maxdeg, const int* sj) -> gevp_status {
    // columns permuted by degree into P1 (F0); F1 = P0; result lands in F0
    zd* F[2] = {P1, P0};
    GEVP_TRY(launch_gather_cols(c, n, nb, P0, n, perm, P1, n));
    for (int j = 1; j <= maxdeg; ++j) {
      const int64_t s0 = sj[j - 1];
      const int64_t cols = nb - s0;
      if (cols <= 0) break;
      info->col_degrees += cols;
      const double* cf = coefs + 3 * (j - 1);
      zd* src = F[(j - 1) & 1];
      zd* dst = F[j & 1];
      GEVP_TRY(fev_mark(c));
      if (j == 1)
        GEVP_TRY(launch_zgemm(c, 0, 0, n, cols, n, 0.0, C, n, src + s0 * n, n, 0.0, src + s0 * n, n,
                              0.0, nullptr, 0, nullptr, dst + s0 * n, n, cf));
      else
        GEVP_TRY(launch_zgemm(c, 0, 0, n, cols, n, 0.0, C, n, src + s0 * n, n, 0.0, src + s0 * n, n,
                              0.0, dst + s0 * n, n, nullptr, dst + s0 * n, n, cf));
      GEVP_TRY(fev_mark(c));
    }
    std::swap(P0, P1);
    return GEVP_OK;
  };

  // Residual-correction filter in low precision (see lanczos_ctl.hip): from
  // the FP64 Ritz pairs (Q = P0, W = C Q, theta) build r' = (W - Q theta)/e and
  // g_1 = r'/theta', run g_{s+1} = a_s (C' g_s + r') - b_s g_{s-1} on the low-
  // precision copy of C, and return Y = Q + g_m in FP64.  Rounding errors are
  // relative to |g|, which shrinks with the residual, so the sweep can reach
  // FP64-level residuals while every filter product is low precision.
  auto run_filter_r2 = [&](int maxdeg, const int* sj, double e_half) -> gevp_status {
    void* F[2] = {G0, G1};
    GEVP_TRY(launch_resid_start32(c, n, nb, W, P0, n, theta, perm, rho0, 1.0 / e_half, Rlp, G1, G0,
                                  n));
    for (int st = 1; st < maxdeg; ++st) {
      const int64_t s0 = sj[st];  // columns with degree >= st + 1
      const int64_t cols = nb - s0;
      if (cols <= 0) break;
      info->col_degrees += cols;
      const double* row = coef2 + (size_t)(st - 1) * 4 * nb;
      char* src = (char*)F[st & 1] + lp_elem * s0 * n;
      char* dst = (char*)F[(st + 1) & 1] + lp_elem * s0 * n;
      char* rr = (char*)Rlp + lp_elem * s0 * n;
      if (bf16) {  // the launcher brackets its product kernel with the event pair
        GEVP_TRY(launch_cgemm_bf16x3_filter(c, n, cols, n, Clp, src, n, dst, n, rr, n, dst, n,
                                            row + s0, row + nb + s0, row + 2 * nb + s0,
                                            row + 3 * nb + s0, bfw));
      } else {
        GEVP_TRY(fev_mark(c));
        GEVP_TRY(launch_cgemm32_filter(c, n, cols, n, Clp, n, src, n, dst, n, rr, n, dst, n,
                                       row + s0, row + nb + s0, row + 2 * nb + s0,
                                       row + 3 * nb + s0));
        GEVP_TRY(fev_mark(c));
      }
    }
    GEVP_TRY(launch_add_correction32(c, n, nb, P0, n, perm, G0, n, P1, n));
    std::swap(P0, P1);
    return GEVP_OK;
  };

  if (need_filter_first) {
    cp.mode = 1;
    GEVP_TRY(launch_control(c, cp, theta, rres, bC, norms, tol, st_i, st_d, perm, coefs));
    GEVP_HIP_TRY(hipMemcpyAsync(hst.data(), st_i, sizeof(int) * hst.size(), hipMemcpyDeviceToHost, c->stream));
    GEVP_HIP_TRY(hipMemcpyAsync(hsd.data(), st_d, sizeof(double) * hsd.size(), hipMemcpyDeviceToHost, c->stream));
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
    tm.start();
    GEVP_TRY(run_filter(hst[1], hst.data() + 4));
    tm.stop(info, GEVP_STAGE_FILTER);
  }
  cp.mode = lp ? 2 : 0;
  bool cfact = false;  // contour factorisations done
  double ca = 0.0, cb = 0.0;
  // Hard locking: every converged wanted Ritz pair leaves the iteration.
  // The filters pass converged (degree-0) columns through unchanged and the
  // degree order puts them first, so after a sweep they are P0's first nl
  // columns; their Ritz values, residuals and W = C P0 columns are permuted
  // to match.  The next sweep projects them out of the active columns (block
  // Gram-Schmidt, twice), orthonormalises and projects only the active ones,
  // and merges the two ascending runs of Ritz values back into one order.
  int64_t nl = 0;
  for (it = 0; it < o.maxit; ++it) {
    const int64_t l0 = (o.lock_mode == 0 && it > 0) ? nl : 0;
    const int64_t na = nb - l0;
    zd* Pa = P0 + l0 * n;
    info->locked = (int)l0;
    tm.start();
    if (l0 > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        GEVP_TRY(launch_zgemm(c, 1, 0, l0, na, n, 1.0, P0, n, Pa, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                              nullptr, Gs, l0));
        GEVP_TRY(launch_zgemm(c, 0, 0, n, na, l0, -1.0, P0, n, Gs, l0, 1.0, Pa, n, 0.0, nullptr, 0,
                              nullptr, Pa, n));
      }
    }
    bool skipped = false;
    GEVP_TRY(cholqr2(c, n, na, Pa, n, qw, &fallbacks, full_seed && it == 0, &skipped));
    if (spec && it == 0) GEVP_HIP_TRY(hipStreamWaitEvent(c->stream, evs.join, 0));
    tm.stop(info, GEVP_STAGE_QR);
    tm.start();
    if (l0 > 0) {
      // Rayleigh-Ritz of the active columns; the locked ones are copied over
      zd* Wa = W + l0 * n;
      GEVP_TRY(launch_zgemm(c, 0, 0, n, na, n, 1.0, C, n, Pa, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, Wa, n));
      GEVP_TRY(launch_zgemm(c, 1, 0, na, na, n, 1.0, Pa, n, Wa, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, Hs, na, nullptr, 1));
      GEVP_TRY(launch_mirror_lower(c, na, Hs, na, Hs, na, nullptr));
      GEVP_TRY(heev_small(c, na, Hs, na, theta + l0, Zs, na, heevw));
      GEVP_TRY(launch_zgemm(c, 0, 0, n, na, na, 1.0, Pa, n, Zs, na, 0.0, nullptr, 0, 0.0, nullptr,
                            0, nullptr, P1 + l0 * n, n));
      GEVP_TRY(launch_zgemm(c, 0, 0, n, na, na, 1.0, Wa, n, Zs, na, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, T + l0 * n, n));
      GEVP_TRY(launch_copy2d(c, n, l0, P0, n, P1, n));
      GEVP_TRY(launch_copy2d(c, n, l0, W, n, T, n));
    } else if (spec && it == 0 && skipped) {
      // Ritz pairs of the seed from the second stream: rotate the basis, then W = C P
      GEVP_TRY(launch_zgemm(c, 0, 0, n, nb, nb, 1.0, P0, n, Zs, nb, 0.0, nullptr, 0, 0.0, nullptr,
                            0, nullptr, P1, n));
      GEVP_TRY(launch_zgemm(c, 0, 0, n, nb, n, 1.0, C, n, P1, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, T, n));
    } else {
      GEVP_TRY(launch_zgemm(c, 0, 0, n, nb, n, 1.0, C, n, P0, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, W, n));
      GEVP_TRY(launch_zgemm(c, 1, 0, nb, nb, n, 1.0, P0, n, W, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, Hs, nb, nullptr, 1));
      GEVP_TRY(launch_mirror_lower(c, nb, Hs, nb, Hs, nb, nullptr));
      GEVP_TRY(heev_small(c, nb, Hs, nb, theta, Zs, nb, heevw));
      GEVP_TRY(launch_zgemm(c, 0, 0, n, nb, nb, 1.0, P0, n, Zs, nb, 0.0, nullptr, 0, 0.0, nullptr,
                            0, nullptr, P1, n));
      GEVP_TRY(launch_zgemm(c, 0, 0, n, nb, nb, 1.0, W, n, Zs, nb, 0.0, nullptr, 0, 0.0, nullptr, 0,
                            nullptr, T, n));
    }
    std::swap(P0, P1);
    std::swap(W, T);
    GEVP_TRY(launch_resid_cols(c, n, na, W + l0 * n, n, P0 + l0 * n, n, theta + l0, rres + l0));
    if (l0 > 0) {
      // one ascending order again: the locked and the active run merged
      GEVP_TRY(launch_merge_runs(c, theta, rres, nb, l0, order));
      GEVP_TRY(launch_gather_cols(c, n, nb, P0, n, order, P1, n));
      GEVP_TRY(launch_gather_cols(c, n, nb, W, n, order, T, n));
      std::swap(P0, P1);
      std::swap(W, T);
    }
    tm.stop(info, GEVP_STAGE_RR);
    info->outer_iters = it + 1;
    if (spec && it == 0) GEVP_HIP_TRY(hipStreamWaitEvent(c->stream, evs.bounds, 0));
    GEVP_TRY(launch_control(c, cp, theta, rres, bC, norms, tol, st_i, st_d, perm, coefs, rho0,
                            coef2));
    GEVP_HIP_TRY(hipMemcpyAsync(hst.data(), st_i, sizeof(int) * hst.size(), hipMemcpyDeviceToHost, c->stream));
    GEVP_HIP_TRY(hipMemcpyAsync(hsd.data(), st_d, sizeof(double) * hsd.size(), hipMemcpyDeviceToHost, c->stream));
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
    info->nconv = hst[0];
    // columns the filter leaves alone (degree 0: the converged wanted ones)
    // are locked for the next sweep
    nl = (!hst[2] && hst[1] > 0) ? hst[4] : 0;
    if (gevp_log_enabled())
      fprintf(stderr, "[gevp] it %d locked %lld nconv %d maxdeg %d a %.4g b %.4g tol %.3g resid %.3g..%.3g\n",
              it, (long long)l0, hst[0], hst[1], hsd[0], hsd[1], hsd[4], hsd[8], hsd[7]);
    if (hst[2]) {
      converged = true;
      break;
    }
    if (it + 1 == o.maxit) break;
    tm.start();
    if (contour) {
      if (!cfact) {
        // circle from the current Ritz values: its right end halfway between
        // the last wanted and the first unwanted one, its left end below the
        // lowest by a twentieth of the width (a small radius separates the
        // wanted from the unwanted faster); factored once per solve
        std::vector<double> th(nb);
        GEVP_HIP_TRY(hipMemcpyAsync(th.data(), theta, sizeof(double) * nb, hipMemcpyDeviceToHost,
                                    c->stream));
        GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
        cb = 0.5 * (th[nev - 1] + th[nev]);
        const double wdt = std::max(cb - th[0], 1e-8 * std::max(1.0, std::fabs(cb)));
        ca = th[0] - 0.05 * wdt;
        if (!(ca < cb) || !std::isfinite(ca) || !std::isfinite(cb)) return GEVP_ERR_NONFINITE;
        int piv = 0;
        if (c32)
          GEVP_TRY(contour_factor32(c, n, C, n, ca, cb, o.nq, cw, nb, &piv));
        else
          GEVP_TRY(contour_factor(c, n, C, n, ca, cb, o.nq, cw, nb, &piv));
        if (piv) return GEVP_ERR_SINGULAR;
        cfact = true;
        info->contour_points = o.nq;
        info->contour_a = ca;
        info->contour_b = cb;
      }
      // only the columns the controller still filters (degree-sorted: the
      // first hst[4] have converged and are kept as they are)
      const int64_t s0 = hst[4];
      GEVP_TRY(launch_gather_cols(c, n, nb, P0, n, perm, P1, n));
      if (s0 > 0) GEVP_TRY(launch_copy2d(c, n, s0, P1, n, P0, n));
      if (s0 < nb && c32) {
        // residuals of the active Ritz pairs (W = C P0 from the Rayleigh-Ritz
        // step) into T, their Ritz values into fres (free until the final stage)
        GEVP_TRY(contour_residual(c, n, nb, s0, perm, W, n, theta, P1, n, T, n, fres));
        GEVP_TRY(contour_apply32(c, n, nb - s0, P1 + s0 * n, n, T + s0 * n, n, fres + s0,
                                 P0 + s0 * n, n, ca, cb, o.nq, cw, nb));
      } else if (s0 < nb) {
        GEVP_TRY(contour_apply(c, n, nb - s0, P1 + s0 * n, n, P0 + s0 * n, n, ca, cb, o.nq, cw, nb));
      }
      info->contour_columns += nb - s0;
      ++info->contour_applications;
    } else if (lp) {
      GEVP_TRY(run_filter_r2(hst[1], hst.data() + 4, hsd[3]));
    } else {
      GEVP_TRY(run_filter(hst[1], hst.data() + 4));
    }
    if (nl > 0) {
      // the columns to lock lead P0 in the filter's degree order: their Ritz
      // values, residuals and C P0 columns follow them
      GEVP_TRY(launch_permute_prefix(c, theta, rres, perm, nl));
      GEVP_TRY(launch_gather_cols(c, n, nl, W, n, perm, T, n));
      std::swap(W, T);
    }
    tm.stop(info, GEVP_STAGE_FILTER);
  }
  info->qr_fallbacks = fallbacks;
  info->filter_flops = 8.0 * (double)n * (double)n * (double)info->col_degrees;

  // ---------------- back-transform and final residuals
  tm.start();
  // Seed monitor in the reduced basis, where both blocks are orthonormal:
  // M = Y0^H Y (= X0^H B X), and the projection residuals R = Y0 - Y M^H of
  // the seed columns onto span(Y) give the sines of the principal angles
  // without the cancellation of k - ||M||_F^2 (sum_j ||r_j||^2 = sum sin^2).
  double hm[5] = {-1.0, -1.0, -1.0, 0.0, -1.0};
  if (monitor) {
    GEVP_TRY(launch_zgemm(c, 1, 0, km, km, n, 1.0, Y0s, n, P0, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, Hs, km));
    GEVP_TRY(launch_zgemm(c, 0, 1, n, km, km, -1.0, P0, n, Hs, km, 1.0, Y0s, n, 0.0, nullptr, 0,
                          nullptr, W, n));
    GEVP_TRY(launch_colnorms(c, n, km, W, n, rmon));
    GEVP_TRY(seed_monitor_stats(c, km, Hs, km, mon, mon + 3 * nb, hm, nullptr, rmon));
    info->seed_sin_rms = hm[0];
    info->seed_dev_mean = hm[1];
    info->seed_dev_max = hm[2];
    info->seed_reindexed = (int)hm[3];
    info->seed_dev_std = hm[4];
  }
  GEVP_TRY(launch_copy2d(c, n, kx, P0, n, X, ldx));
  GEVP_TRY(trsm_left_lower_c(c, n, kx, L, n, Dinv, n, X, ldx, 1));
  GEVP_TRY(launch_phase_normalize(c, n, kx, X, ldx));
  GEVP_TRY(launch_copy_real(c, kx, theta, lambda));
  double hn[2] = {0.0, 0.0};
  GEVP_HIP_TRY(hipMemcpyAsync(hn, norms, sizeof(hn), hipMemcpyDeviceToHost, c->stream));
  if (!o.skip_final) {
    // R = A X - B X diag(lambda) for the nev wanted columns (all kx when the
    // caller asks for the residuals): [A X; B X] as one 2n-row product (its
    // tiles fill the compute units' rounds better than two n-row products),
    // then the column norms of the top half minus the scaled bottom half
    const int64_t kr = resid_out ? kx : nev;
    GEVP_TRY(launch_zgemm(c, 0, 0, 2 * n, kr, n, 1.0, Af, n, X, ldx, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, WT, 2 * n, nullptr, 0, 0, n, Bf));
    GEVP_TRY(launch_resid_cols(c, n, kr, WT, 2 * n, WT + n, 2 * n, theta, fres));
    if (resid_out) GEVP_TRY(launch_copy_real(c, kx, fres, resid_out));
    std::vector<double> hr(kr);
    GEVP_HIP_TRY(hipMemcpyAsync(hr.data(), fres, sizeof(double) * kr, hipMemcpyDeviceToHost, c->stream));
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
    double mx = 0.0;
    for (int64_t i = 0; i < nev; ++i) mx = std::max(mx, hr[i]);
    info->max_resid = (hn[0] > 0.0) ? mx / hn[0] : mx;
    if (converged && info->max_resid > tol) st = GEVP_ERR_NOCONV;
  } else {
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
  }
  tm.stop(info, GEVP_STAGE_FINAL);
  GEVP_TRY(fev_collect(c, info));
  // the second and the panel stream joined the main stream before its final
  // synchronisation, so their events have completed too
  GEVP_TRY(gev_collect(c, info));
  if (c->inner_streams) {
    GEVP_TRY(gev_collect(c->aux, info));
    GEVP_TRY(gev_collect(c->panel, info));
  }
  info->normA = hn[0];
  info->normB = hn[1];
  if (!converged) st = GEVP_ERR_NOCONV;
  if (st == GEVP_ERR_NOCONV) info->lapack_info = nev - info->nconv;
  return st;
}

gevp_status gevp_backward(gevp_handle h, int64_t n, int64_t nev, const void* X_, int64_t ldx,
                          const double* lambda, const double* w, void* dA_, int64_t ldda, void* dB_,
                          int64_t lddb) {
  if (!h || n < 1 || nev < 1 || nev > n || !X_ || ldx < n || !w) return GEVP_ERR_INVALID;
  if (dA_ && ldda < n) return GEVP_ERR_INVALID;
  if (dB_ && (lddb < n || !lambda)) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  gevp_ctx* c = h;
  const zd* X = (const zd*)X_;
  const size_t need = ws_round(sizeof(zd) * n * nev) + ws_round(sizeof(double) * nev);
  GEVP_TRY(ws_reserve(c, need));
  zd* Xw = (zd*)ws_take(c, sizeof(zd) * n * nev);
  if (dA_) {
    GEVP_TRY(launch_scale_cols(c, n, nev, X, ldx, w, Xw, n));
    GEVP_TRY(launch_zgemm(c, 0, 1, n, n, nev, 1.0, Xw, n, X, ldx, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, (zd*)dA_, ldda));
  }
  if (dB_) {
    double* wl = (double*)ws_take(c, sizeof(double) * nev);
    (void)wl;
    // dB = -X diag(w lambda) X^H: scale by w, then by lambda with alpha = -1
    GEVP_TRY(launch_scale_cols(c, n, nev, X, ldx, w, Xw, n));
    GEVP_TRY(launch_scale_cols(c, n, nev, Xw, n, lambda, Xw, n));
    GEVP_TRY(launch_zgemm(c, 0, 1, n, n, nev, -1.0, Xw, n, X, ldx, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, (zd*)dB_, lddb));
  }
  return GEVP_OK;
}

gevp_status gevp_backward_noalloc(gevp_handle h, int64_t n, int64_t nev, const void* X_,
                                  int64_t ldx, const double* lambda, const double* w, void* dA_,
                                  int64_t ldda, void* dB_, int64_t lddb) {
  if (!h || n < 1 || nev < 1 || nev > n || !X_ || ldx < n || !w) return GEVP_ERR_INVALID;
  if (dA_ && ldda < n) return GEVP_ERR_INVALID;
  if (dB_ && (lddb < n || !lambda)) return GEVP_ERR_INVALID;
  if ((size_t)n * (size_t)nev * sizeof(zd) > SCRATCH_BYTES) return GEVP_ERR_WORKSPACE;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  void* sp = nullptr;
  GEVP_TRY(scratch_address(h->device, &sp));  // looked up by gevp_create already
  gevp_ctx* c = h;
  const zd* X = (const zd*)X_;
  zd* Xw = (zd*)sp;  // n x nev scaled columns, in the scratch array
  // no split-K buffer and no profiling events for the duration of the call
  const bool ns = c->no_split;
  const int prof = c->profiling;
  c->no_split = true;
  c->profiling = 0;
  gevp_status st = GEVP_OK;
  if (dA_) {
    st = launch_scale_cols(c, n, nev, X, ldx, w, Xw, n);
    if (st == GEVP_OK)
      st = launch_zgemm(c, 0, 1, n, n, nev, 1.0, Xw, n, X, ldx, 0.0, nullptr, 0, 0.0, nullptr, 0,
                        nullptr, (zd*)dA_, ldda);
  }
  if (st == GEVP_OK && dB_) {
    st = launch_scale_cols(c, n, nev, X, ldx, w, Xw, n);
    if (st == GEVP_OK) st = launch_scale_cols(c, n, nev, Xw, n, lambda, Xw, n);
    if (st == GEVP_OK)
      st = launch_zgemm(c, 0, 1, n, n, nev, -1.0, Xw, n, X, ldx, 0.0, nullptr, 0, 0.0, nullptr, 0,
                        nullptr, (zd*)dB_, lddb);
  }
  c->no_split = ns;
  c->profiling = prof;
  return st;
}

gevp_status gevp_solve_batched(gevp_handle h, const gevp_opts* opts, int count, const int64_t* n,
                               const void* const* A, const int64_t* lda, const void* const* B,
                               const int64_t* ldb, const void* const* X0, const int64_t* ldx0,
                               const int64_t* k0, const int64_t* nev, double tol,
                               const int64_t* kx, double* const* lambda, void* const* X,
                               const int64_t* ldx, double* const* resid, gevp_info* infos) {
  if (!h || count < 0 || !n || !A || !lda || !B || !ldb || !nev || !lambda || !X || !ldx)
    return GEVP_ERR_INVALID;
  if (count == 0) return GEVP_OK;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  int streams = batch_stream_count(opts, count);
  if (h->tune_streams > 0 && !h->ext) streams = std::min(std::min(h->tune_streams, 16), count);
  while ((int)h->workers.size() < streams) {
    gevp_ctx* w = new gevp_ctx();
    w->device = h->device;
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      return GEVP_ERR_HIP;
    }
    w->owns_stream = true;
    w->inner_streams = false;
    h->workers.push_back(w);
  }
  // event timing of the filter launches (profiling flag 2) carries over; the
  // per-stage timer (flag 1) would synchronise the workers and is not passed on
  for (int w = 0; w < streams; ++w) {
    gevp_ctx* c = h->workers[w];
    c->profiling = h->profiling & 6;
    c->no_split = h->tune_split == 2;
    c->cu_div = h->tune_split == 1 ? streams : 1;
  }
  if (h->ext) {
    // caller-owned memory: worker w takes the w-th equal share, its solve
    // workspace first and its split-K buffer at the share's top end
    const size_t per = worker_share(h, streams);
    if (per <= SKW_BYTES + 256) return GEVP_ERR_WORKSPACE;
    for (int w = 0; w < streams; ++w) {
      gevp_ctx* c = h->workers[w];
      char* base = h->ext_base + (size_t)w * per;
      c->ext = true;
      c->ws = base;
      c->ws_bytes = per - SKW_BYTES;
      c->ws_used = 0;
      c->skw = base + per - SKW_BYTES;
      c->skw_bytes = SKW_BYTES;
    }
  }
  // the worker streams start after the work already queued on the caller's stream
  hipEvent_t ready;
  GEVP_HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  GEVP_HIP_TRY(hipEventRecord(ready, h->stream));
  for (int w = 0; w < streams; ++w) GEVP_HIP_TRY(hipStreamWaitEvent(h->workers[w]->stream, ready, 0));
  // largest problems first (cost ~ n^3)
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  std::vector<gevp_status> st(count, GEVP_OK);
  std::atomic<int> next(0);
  auto work = [&](int w) {
    gevp_ctx* c = h->workers[w];
    (void)hipSetDevice(c->device);
    for (;;) {
      const int q = next.fetch_add(1);
      if (q >= count) break;
      const int i = order[q];
      const void* x0 = X0 ? X0[i] : nullptr;
      st[i] = gevp_solve(c, opts, n[i], A[i], lda[i], B[i], ldb[i], x0, ldx0 ? ldx0[i] : n[i],
                         (k0 && x0) ? k0[i] : 0, nev[i], tol, kx ? kx[i] : nev[i], lambda[i], X[i],
                         ldx[i], resid ? resid[i] : nullptr, infos ? infos + i : nullptr);
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < streams; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto& t : pool) t.join();
  (void)hipEventDestroy(ready);
  gevp_status worst = GEVP_OK;
  for (int i = 0; i < count; ++i) {
    const gevp_status s = st[i];
    if (s == GEVP_OK) continue;
    if (worst == GEVP_OK || worst == GEVP_ERR_NOCONV) worst = s;
  }
  return worst;
}

gevp_status gevp_set_tuning(gevp_handle h, const gevp_tuning* t) {
  if (!h) return GEVP_ERR_INVALID;
  if (!t) {
    h->tune_streams = 0;
    h->tune_split = 0;
    h->tune_seconds = 0.0;
    return GEVP_OK;
  }
  if (t->streams < 0 || t->streams > 16 || t->split_mode < 0 || t->split_mode > 2)
    return GEVP_ERR_INVALID;
  h->tune_streams = t->streams;
  h->tune_split = t->split_mode;
  h->tune_seconds = t->seconds;
  return GEVP_OK;
}

gevp_status gevp_get_tuning(gevp_handle h, gevp_tuning* t) {
  if (!h || !t) return GEVP_ERR_INVALID;
  *t = gevp_tuning{};
  t->streams = h->tune_streams;
  t->split_mode = h->tune_split;
  t->seconds = h->tune_seconds;
  return GEVP_OK;
}

gevp_status gevp_autotune_batched(gevp_handle h, const gevp_opts* opts, int count,
                                  const int64_t* n, const void* const* A, const int64_t* lda,
                                  const void* const* B, const int64_t* ldb,
                                  const void* const* X0, const int64_t* ldx0, const int64_t* k0,
                                  const int64_t* nev, double tol, const int64_t* kx,
                                  double* const* lambda, void* const* X, const int64_t* ldx,
                                  double* const* resid, gevp_tuning* best) {
  if (!h || count < 1) return GEVP_ERR_INVALID;
  std::vector<int> cand;
  for (int s : {4, 8, 12, 16})
    if (s <= count) cand.push_back(s);
  if (count < 16 && std::find(cand.begin(), cand.end(), count) == cand.end()) cand.push_back(count);
  const int save_s = h->tune_streams, save_m = h->tune_split;
  const double save_t = h->tune_seconds;
  auto call = [&]() {
    return gevp_solve_batched(h, opts, count, n, A, lda, B, ldb, X0, ldx0, k0, nev, tol, kx, lambda,
                              X, ldx, resid, nullptr);
  };
  auto restore = [&]() {
    h->tune_streams = save_s;
    h->tune_split = save_m;
    h->tune_seconds = save_t;
  };
  // untimed: every worker stream and workspace the candidates need
  h->tune_streams = cand.back();
  h->tune_split = 0;
  gevp_status st = call();
  if (st != GEVP_OK && st != GEVP_ERR_NOCONV) {
    restore();
    return st;
  }
  int bs = 0, bm = 0;
  double bt = 0.0;
  for (int s : cand)
    for (int m = 0; m < 3; ++m) {
      h->tune_streams = s;
      h->tune_split = m;
      GEVP_HIP_TRY(hipDeviceSynchronize());
      const auto t0 = std::chrono::steady_clock::now();
      st = call();
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (st != GEVP_OK && st != GEVP_ERR_NOCONV) {
        restore();
        return st;
      }
      if (bs == 0 || dt < bt) {
        bs = s;
        bm = m;
        bt = dt;
      }
    }
  h->tune_streams = bs;
  h->tune_split = bm;
  h->tune_seconds = bt;
  if (best) GEVP_TRY(gevp_get_tuning(h, best));
  return st;
}

// ---- kernel-level entry points

gevp_status gevp_k_zgemm(gevp_handle h, char opA, char opB, int64_t m, int64_t n, int64_t k,
                         double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                         double beta, const void* Cm, int64_t ldc, double gamma, const void* E,
                         int64_t lde, const double* gcol, void* D, int64_t ldd) {
  if (!h || m < 0 || n < 0 || k < 0 || !D) return GEVP_ERR_INVALID;
  const int oa = (opA == 'C' || opA == 'c') ? 1 : 0;
  const int ob = (opB == 'C' || opB == 'c') ? 1 : 0;
  if (!(opA == 'N' || opA == 'n' || oa) || !(opB == 'N' || opB == 'n' || ob)) return GEVP_ERR_INVALID;
  if (k > 0 && (!A || !B)) return GEVP_ERR_INVALID;
  if (k > 0 && lda < (oa ? k : m)) return GEVP_ERR_INVALID;
  if (k > 0 && ldb < (ob ? n : k)) return GEVP_ERR_INVALID;
  if (ldd < m || (Cm && ldc < m) || (E && lde < m)) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  return launch_zgemm(h, oa, ob, m, n, k, alpha, (const zd*)A, lda, (const zd*)B, ldb, beta,
                      (const zd*)Cm, ldc, gamma, (const zd*)E, lde, gcol, (zd*)D, ldd);
}

gevp_status gevp_k_zgemm_tri(gevp_handle h, char opA, char opB, int64_t m, int64_t n, int64_t k,
                             double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                             double beta, const void* Cm, int64_t ldc, void* D, int64_t ldd,
                             int lower, int upperA) {
  if (!h || m < 0 || n < 0 || k < 0 || !D) return GEVP_ERR_INVALID;
  if ((lower != 0 && lower != 1) || (upperA != 0 && upperA != 1) || (lower && m != n))
    return GEVP_ERR_INVALID;
  const int oa = (opA == 'C' || opA == 'c') ? 1 : 0;
  const int ob = (opB == 'C' || opB == 'c') ? 1 : 0;
  if (!(opA == 'N' || opA == 'n' || oa) || !(opB == 'N' || opB == 'n' || ob)) return GEVP_ERR_INVALID;
  if (k > 0 && (!A || !B)) return GEVP_ERR_INVALID;
  if (k > 0 && lda < (oa ? k : m)) return GEVP_ERR_INVALID;
  if (k > 0 && ldb < (ob ? n : k)) return GEVP_ERR_INVALID;
  if (ldd < m || (Cm && ldc < m)) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  return launch_zgemm(h, oa, ob, m, n, k, alpha, (const zd*)A, lda, (const zd*)B, ldb, beta,
                      (const zd*)Cm, ldc, 0.0, nullptr, 0, nullptr, (zd*)D, ldd, nullptr, lower,
                      upperA);
}

gevp_status gevp_k_filter_gemm(gevp_handle h, int precision, int64_t n, int64_t m,
                               const void* C, int64_t ldc, const void* G, int64_t ldg,
                               const void* P, int64_t ldp, const void* R, int64_t ldr, void* D,
                               int64_t ldd, const double* alpha, const double* beta,
                               const double* gamma, const double* delta) {
  if (!h || n < 1 || m < 0 || !C || ldc < n || !G || ldg < n || !P || ldp < n || !R || ldr < n ||
      !D || ldd < n || !alpha || !beta || !gamma || !delta)
    return GEVP_ERR_INVALID;
  if (precision != GEVP_FP32 && precision != GEVP_BF16X3) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  const bool bf = precision == GEVP_BF16X3;
  const size_t bytes = bf ? bf16_planes_bytes(n) : (size_t)8 * n * n;
  const size_t wbytes = bf ? bf16_filter_work_bytes(n, m) : 0;
  GEVP_TRY(ws_reserve(h, ws_round(bytes) + wbytes));
  void* planes = ws_take(h, bytes);
  if (bf) {
    void* work = ws_take(h, wbytes);
    GEVP_TRY(launch_split_rows_bf16(h, n, (const zd*)C, ldc, planes));
    return launch_cgemm_bf16x3_filter(h, n, m, n, planes, G, ldg, P, ldp, R, ldr, D, ldd, alpha, beta,
                                      gamma, delta, work);
  }
  GEVP_TRY(launch_to_c32(h, n, n, (const zd*)C, ldc, planes, n));
  return launch_cgemm32_filter(h, n, m, n, planes, n, G, ldg, P, ldp, R, ldr, D, ldd, alpha, beta,
                               gamma, delta);
}

gevp_status gevp_k_hemv(gevp_handle h, int64_t n, const void* M, int64_t ldm, const void* x, void* y) {
  if (!h || n < 1 || !M || ldm < n || !x || !y) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  GEVP_TRY(ws_reserve(h, hemv_work_bytes(n) + 256));
  void* w = ws_take(h, hemv_work_bytes(n));
  return launch_hemv(h, n, (const zd*)M, ldm, (const zd*)x, (zd*)y, w);
}

gevp_status gevp_k_potrf(gevp_handle h, int64_t n, void* M, int64_t ldm, int64_t* pivot) {
  if (!h || n < 1 || !M || ldm < n) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  GEVP_TRY(ws_reserve(h, ws_round(sizeof(zd) * n * 64) + 256));
  zd* Dinv = (zd*)ws_take(h, sizeof(zd) * n * 64);
  int* flag = (int*)ws_take(h, sizeof(int) * 4);
  const int big = 0x7fffffff;
  GEVP_HIP_TRY(hipMemcpyAsync(flag, &big, sizeof(int), hipMemcpyHostToDevice, h->stream));
  GEVP_TRY(chol_lower(h, n, (zd*)M, ldm, Dinv, n, flag));
  int f = big;
  GEVP_HIP_TRY(hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(h->stream));
  if (pivot) *pivot = (f == big) ? 0 : f;
  return (f == big) ? GEVP_OK : GEVP_ERR_NOT_HPD;
}

gevp_status gevp_k_trsm(gevp_handle h, char side, char trans, int64_t n, int64_t m, const void* L,
                        int64_t ldl, void* R, int64_t ldr) {
  if (!h || n < 1 || m < 0 || !L || ldl < n || !R) return GEVP_ERR_INVALID;
  const bool left = (side == 'L' || side == 'l');
  const bool conj = (trans == 'C' || trans == 'c');
  if (!left && !(side == 'R' || side == 'r')) return GEVP_ERR_INVALID;
  if (!conj && !(trans == 'N' || trans == 'n')) return GEVP_ERR_INVALID;
  if (!left && !conj) return GEVP_ERR_INVALID;
  if (ldr < (left ? n : m)) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  // the diagonal-block inverses come from re-factoring a copy of L L^H's
  // diagonal blocks: L's own diagonal blocks are inverted directly instead
  GEVP_TRY(ws_reserve(h, ws_round(sizeof(zd) * n * 64) + ws_round(sizeof(zd) * n * n) + 256));
  zd* Dinv = (zd*)ws_take(h, sizeof(zd) * n * 64);
  zd* Lc = (zd*)ws_take(h, sizeof(zd) * n * n);
  GEVP_TRY(launch_copy2d(h, n, n, (const zd*)L, ldl, Lc, n));
  GEVP_TRY(diag_block_inverses(h, n, Lc, n, Dinv, n));
  if (left && !conj) return trsm_left_lower_n(h, n, m, Lc, n, Dinv, n, (zd*)R, ldr);
  if (left && conj) return trsm_left_lower_c(h, n, m, Lc, n, Dinv, n, (zd*)R, ldr);
  return trsm_right_lower_c(h, n, m, Lc, n, Dinv, n, (zd*)R, ldr);
}

gevp_status gevp_k_seed_monitor(gevp_handle h, int64_t k, const void* M, int64_t ldm, double* stats,
                                int* match) {
  if (!h || k < 1 || k > 8192 || !M || ldm < k || !stats) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  const size_t sb = sizeof(double) * 6 * (k + 1);  // matching work arrays beyond the LDS limit
  GEVP_TRY(ws_reserve(h, ws_round(sizeof(double) * (3 * k + 8)) + ws_round(sb) + 512));
  double* w = (double*)ws_take(h, sizeof(double) * (3 * k + 8));
  void* s = ws_take(h, sb);
  return seed_monitor_stats(h, k, (const zd*)M, ldm, w, w + 3 * k, stats, match, nullptr, s, sb);
}

gevp_status gevp_k_heev(gevp_handle h, int64_t n, void* H, int64_t ldh, double* theta, void* Z,
                        int64_t ldz) {
  if (!h || n < 1 || n > 2048 || !H || ldh < n || !theta || !Z || ldz < n) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  GEVP_TRY(ws_reserve(h, heev_work_bytes(n) + ws_round(sizeof(zd) * n * n) + 256));
  void* w = ws_take(h, heev_work_bytes(n));
  zd* Hf = (zd*)ws_take(h, sizeof(zd) * n * n);
  int* flag = (int*)ws_take(h, sizeof(int) * 4);
  GEVP_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), h->stream));
  GEVP_TRY(launch_mirror_lower(h, n, (const zd*)H, ldh, Hf, n, flag));
  GEVP_TRY(heev_small(h, n, Hf, n, theta, (zd*)Z, ldz, w));
  GEVP_HIP_TRY(hipStreamSynchronize(h->stream));
  return GEVP_OK;
}

}  // extern "C"
