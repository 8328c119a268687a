// Host side of libbatched_omp.so: argument validation, the layouts of the
// prepared dictionary and of the workspace, and the iteration driver that
// enqueues the kernels of one batched OMP solve (Algorithm 1 for every signal).
//
// Every argument check runs on the host before anything is enqueued; a
// negative return therefore leaves the stream untouched (OMP_EDEVICE aside).

#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/batched_omp.h"
#include "omp_internal.h"

namespace bomp {
namespace {

thread_local int g_last_hip_error = 0;

constexpr size_t ALIGN = 256;

struct Carve {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    const size_t at = off;
    off += count * sizeof(T);
    return at;
  }
};

struct DictLayout {
  int64_t Mp, Np;
  size_t nu2, inv_nu, A32, G, A16, aerr, aerr_max, G64, inv_nu64, inv_nu_h, total;
};

DictLayout dict_layout(int64_t M, int64_t N, int precision) {
  DictLayout L;
  L.Mp = round_up(M, KPAD);
  L.Np = round_up(N, NPAD);
  Carve c;
  L.nu2 = c.take<double>(L.Np);
  L.inv_nu = c.take<float>(L.Np);
  L.A32 = c.take<float>((size_t)L.Np * L.Mp);
  L.G = c.take<float>((size_t)L.Np * L.Np);
  L.A16 = is_half(precision) ? c.take<uint16_t>((size_t)L.Np * L.Mp) : 0;
  L.aerr = c.take<float>(L.Np);
  L.aerr_max = c.take<float>(1);
  L.G64 = precision == OMP_PREC_FP64 ? c.take<double>((size_t)L.Np * L.Np) : 0;
  L.inv_nu64 = precision == OMP_PREC_FP64 ? c.take<double>(L.Np) : 0;
  L.inv_nu_h = precision == OMP_PREC_FP16 ? c.take<float>(L.Np) : 0;
  L.total = (c.off + ALIGN - 1) / ALIGN * ALIGN;
  return L;
}

struct WorkLayout {
  int64_t Mp, Np, Bp;
  CorrGeom g;
  int ntile;
  int nslice, slice_len;
  int64_t vstride;
  size_t Yp, R32, R16, part, mask, k, flags, pnorm, pdelta, Sb, epsb, sup, u, xh, V, P, Pk, D, P64, D64, V64, u64,
      rscale, rscale_next, total;
  int pchunks;
};

WorkLayout work_layout(int64_t M, int64_t N, int64_t B, int S, int precision, int cfg, bool gram_dom = false,
                       bool ties = false, bool v0 = false) {
  WorkLayout L;
  L.Mp = round_up(M, KPAD);
  L.Np = round_up(N, NPAD);
  L.Bp = round_up(B > 0 ? B : 1, BPAD);
  L.g = corr_geometry(precision, L.Np, L.Bp, cfg, ties);
  L.ntile = (int)(L.Np / L.g.tile_atoms);
  // Slice the residual over the XCDs when the FP32 dictionary outgrows one L2.
  L.nslice = (L.Np * L.Mp * 4 > (int64_t)2 << 20) ? NSLICE_MAX : 1;
  L.slice_len = (int)(L.Mp / L.nslice);
  const size_t Bp = (size_t)L.Bp, Sz = (size_t)S;
  Carve c;
  L.Yp = c.take<float>(Bp * L.Mp);
  L.R32 = c.take<float>(Bp * L.Mp);
  L.R16 = is_half(precision) ? c.take<uint16_t>(Bp * L.Mp) : 0;
  L.rscale = precision == OMP_PREC_FP16 ? c.take<float>(Bp) : 0;
  L.rscale_next = precision == OMP_PREC_FP16 ? c.take<float>(Bp) : 0;
  // (the Gram-domain select writes GSLICE keys per signal, twice that with near-tie flagging)
  // (the Gram-domain select writes GSLICE keys per signal, twice that with near-tie
  // flagging; v0 two keys, the FP64 form two (score, index) pairs of doubles)
  L.part = c.take<uint64_t>(Bp * (size_t)std::max<int64_t>((int64_t)L.ntile * L.g.keys_per_tile,
                                                            gram_dom ? GSLICE * (ties ? 2 : 1) : 4));
  L.mask = c.take<uint32_t>(Bp * (L.Np / 32));
  L.k = c.take<int32_t>(Bp);
  L.flags = c.take<int32_t>(Bp);
  L.pnorm = c.take<double>(Bp * NSLICE_MAX);
  L.pdelta = c.take<double>(Bp * NSLICE_MAX);
  L.Sb = c.take<int32_t>(Bp);
  L.epsb = c.take<float>(Bp);
  L.sup = c.take<int32_t>(Bp * Sz);
  L.u = c.take<float>(Bp * Sz);
  L.xh = c.take<float>(Bp * Sz);
  L.vstride = round_up((int64_t)(Sz * (Sz + 1) / 2), 4);
  L.V = c.take<float>(Bp * (size_t)L.vstride);
  const bool f64 = precision == OMP_PREC_FP64;  // the FP64 form (v0 in FP64)
  const bool proj = (gram_dom || v0) && !f64;   // FP32 forms that start from P = A^T y
  L.P = proj ? c.take<float>(Bp * (size_t)L.Np) : 0;
  L.pchunks = proj ? project_chunks(L.Bp, L.Np, L.Mp) : 1;
  L.Pk = L.pchunks > 1 ? c.take<float>((size_t)L.pchunks * Bp * (size_t)L.Np) : 0;
  L.D = (v0 && !f64) ? c.take<float>(Bp * Sz * (size_t)L.Np) : 0;
  L.P64 = f64 ? c.take<double>(Bp * (size_t)L.Np) : 0;
  L.D64 = f64 ? c.take<double>(Bp * Sz * (size_t)L.Np) : 0;
  L.V64 = f64 ? c.take<double>(Bp * (size_t)L.vstride) : 0;
  L.u64 = f64 ? c.take<double>(Bp * Sz) : 0;
  L.total = (c.off + ALIGN - 1) / ALIGN * ALIGN;
  return L;
}

template <class T>
T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

}  // namespace

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool valid_precision(int p) {
  return p == OMP_PREC_FP32 || p == OMP_PREC_BF16 || p == OMP_PREC_FP64 || p == OMP_PREC_FP16;
}

// Sizes whose padded buffers would overflow or exceed any real device are rejected.
bool dims_ok(int64_t M, int64_t N) {
  return M >= 1 && N >= 1 && M <= (int64_t)1 << 24 && N <= (int64_t)1 << 20;
}

int device_error(hipError_t e) {
  g_last_hip_error = (int)e;
  return OMP_EDEVICE;
}

// The library is built for gfx950 only; refuse any other device up front.
int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e);
  static std::mutex mu;
  static std::vector<int> ok;  // per device: 0 unknown, 1 gfx950, -1 other
  std::lock_guard<std::mutex> lock(mu);
  if ((int)ok.size() <= dev) ok.resize(dev + 1, 0);
  if (ok[dev] == 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return device_error(e);
    ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
  }
  if (ok[dev] < 0) {
    g_last_hip_error = (int)hipErrorInvalidDeviceFunction;
    return OMP_EDEVICE;
  }
  return OMP_OK;
}

namespace {

// Optional profiling (omp_opts_t.phase_ms): brackets every launch with a pair
// of hipEvents on the solve's stream and sums the elapsed times per phase. The
// events come from a per-thread pool that is created once and reused, so that
// timing adds no event creation to the enqueue path (which would otherwise let
// the GPU run ahead of the host and idle between launches).
class PhaseTimer {
 public:
  PhaseTimer(float *ms, int32_t *launches, hipStream_t st) : ms_(ms), n_(launches), st_(st) {}
  bool on() const { return ms_ != nullptr; }
  void reset() {
    used_ = 0;
    phases_.clear();
  }
  template <class F>
  hipError_t run(int phase, F &&launch) {
    if (!ms_) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = pool_get(2 * used_, &a);
    if (e == hipSuccess) e = pool_get(2 * used_ + 1, &b);
    if (e == hipSuccess) e = hipEventRecord(a, st_);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, st_);
    if (e == hipSuccess) {
      phases_.push_back(phase);
      ++used_;
    }
    return e;
  }
  hipError_t finish() {
    if (!ms_) return hipSuccess;
    hipError_t e = hipStreamSynchronize(st_);
    for (int p = 0; p < OMP_NPHASE; ++p) {
      ms_[p] = 0.f;
      if (n_) n_[p] = 0;
    }
    for (size_t i = 0; i < used_ && e == hipSuccess; ++i) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, pool()[2 * i], pool()[2 * i + 1]);
      ms_[phases_[i]] += t;
      if (n_) n_[phases_[i]] += 1;
    }
    return e;
  }

 private:
  // Held until the process ends (never destroyed: the runtime may already be
  // shutting down when thread-local destructors run).
  static std::vector<hipEvent_t> &pool() {
    thread_local std::vector<hipEvent_t> *ev = new std::vector<hipEvent_t>();
    return *ev;
  }
  static hipError_t pool_get(size_t i, hipEvent_t *out) {
    std::vector<hipEvent_t> &ev = pool();
    while (ev.size() <= i) {
      hipEvent_t x = nullptr;
      hipError_t e = hipEventCreate(&x);
      if (e != hipSuccess) return e;
      ev.push_back(x);
    }
    *out = ev[i];
    return hipSuccess;
  }
  float *ms_;
  int32_t *n_;
  hipStream_t st_;
  size_t used_ = 0;
  std::vector<int> phases_;
};

}  // namespace

size_t dict_bytes(int64_t M, int64_t N, int precision) { return dict_layout(M, N, precision).total; }

DictView dict_view(void *mem, int64_t M, int64_t N, int precision) {
  const DictLayout L = dict_layout(M, N, precision);
  DictView d;
  d.M = M;
  d.N = N;
  d.Mp = L.Mp;
  d.Np = L.Np;
  d.nu2 = at<double>(mem, L.nu2);
  d.inv_nu = at<float>(mem, L.inv_nu);
  d.A32 = at<float>(mem, L.A32);
  d.G = at<float>(mem, L.G);
  d.A16 = is_half(precision) ? at<uint16_t>(mem, L.A16) : nullptr;
  d.inv_nu_h = precision == OMP_PREC_FP16 ? at<float>(mem, L.inv_nu_h) : nullptr;
  d.aerr = at<float>(mem, L.aerr);
  d.aerr_max = at<float>(mem, L.aerr_max);
  d.G64 = precision == OMP_PREC_FP64 ? at<double>(mem, L.G64) : nullptr;
  d.inv_nu64 = precision == OMP_PREC_FP64 ? at<double>(mem, L.inv_nu64) : nullptr;
  return d;
}

size_t work_bytes(int64_t M, int64_t N, int64_t B, int S, int precision, int cfg, bool gram_dom, bool ties,
                  bool v0) {
  return work_layout(M, N, B, S, precision, cfg, gram_dom, ties, v0).total;
}

bool solve_fits(int64_t M, int64_t N, int64_t B, int S, int precision, int cfg) {
  const WorkLayout L = work_layout(M, N, B, S, precision, cfg);
  return solve_waves_for(L.vstride, L.ntile * L.g.keys_per_tile, is_half(precision)) > 0;
}

WorkView work_view(void *mem, int64_t M, int64_t N, int64_t B, int S, int precision, int cfg, bool gram_dom,
                   bool ties, bool v0) {
  const WorkLayout L = work_layout(M, N, B, S, precision, cfg, gram_dom, ties, v0);
  WorkView w;
  w.B = B;
  w.Bp = L.Bp;
  w.Mp = L.Mp;
  w.Np = L.Np;
  w.S = S;
  w.tile_cfg = L.g.cfg;
  w.ntile = L.ntile;
  w.ncand = L.g.keys_per_tile;
  w.tile_atoms = L.g.tile_atoms;
  w.wave_atoms = L.g.wave_atoms;
  w.sub_frags = L.g.sub_frags;
  w.subs_per_half = L.g.subs_per_half;
  w.Yp = at<float>(mem, L.Yp);
  w.R32 = at<float>(mem, L.R32);
  w.R16 = is_half(precision) ? at<uint16_t>(mem, L.R16) : nullptr;
  w.fp16 = precision == OMP_PREC_FP16 ? 1 : 0;
  w.rscale = L.rscale ? at<float>(mem, L.rscale) : nullptr;
  w.rscale_next = L.rscale_next ? at<float>(mem, L.rscale_next) : nullptr;
  w.part = at<uint64_t>(mem, L.part);
  w.mask = at<uint32_t>(mem, L.mask);
  w.k = at<int32_t>(mem, L.k);
  w.flags = at<int32_t>(mem, L.flags);
  w.pnorm = at<double>(mem, L.pnorm);
  w.pdelta = at<double>(mem, L.pdelta);
  w.vstride = L.vstride;
  w.nslice = L.nslice;
  w.slice_len = L.slice_len;
  w.Sb = at<int32_t>(mem, L.Sb);
  w.epsb = at<float>(mem, L.epsb);
  w.sup = at<int32_t>(mem, L.sup);
  w.u = at<float>(mem, L.u);
  w.xh = at<float>(mem, L.xh);
  w.V = at<float>(mem, L.V);
  w.gram_fly = 0;
  w.refactor = 0;
  w.gram_dom = gram_dom ? 1 : 0;
  const bool f64 = precision == OMP_PREC_FP64;
  w.P = L.P ? at<float>(mem, L.P) : nullptr;
  w.v0 = (v0 || f64) ? 1 : 0;
  w.D = L.D ? at<float>(mem, L.D) : nullptr;
  w.P64 = f64 ? at<double>(mem, L.P64) : nullptr;
  w.D64 = f64 ? at<double>(mem, L.D64) : nullptr;
  w.V64 = f64 ? at<double>(mem, L.V64) : nullptr;
  w.u64 = f64 ? at<double>(mem, L.u64) : nullptr;
  w.pchunks = L.pchunks;
  w.Pk = L.pchunks > 1 ? at<float>(mem, L.Pk) : nullptr;
  w.flag_ties = ties ? 1 : 0;
  w.fuse_res = 0;
  if (gram_dom) {  // one key (two with near-tie flagging) per (signal, atom slice) from the Gram-domain select
    w.ntile = GSLICE;
    w.ncand = ties ? 2 : 1;
  }
  return w;
}

}  // namespace bomp

using namespace bomp;

extern "C" {

const char *omp_version(void) { return "0.1.0"; }

const char *omp_status_string(int status) {
  switch (status) {
    case OMP_OK: return "ok";
    case OMP_EINVAL: return "invalid argument";
    case OMP_EWORKSPACE: return "workspace or dictionary memory missing, too small or misaligned";
    case OMP_EDEVICE: return "HIP runtime error or unsupported device (needs gfx950)";
    case OMP_ENOTSUPP: return "request exceeds the library's limits";
    default: return "unknown status";
  }
}

int omp_last_hip_error(void) { return g_last_hip_error; }

void omp_opts_default(omp_opts_t *opts) {
  if (!opts) return;
  std::memset(opts, 0, sizeof(*opts));
  opts->precision = OMP_PREC_FP32;
  opts->use_graph = 1;
}

size_t omp_dict_size(int64_t M, int64_t N, int32_t precision) {
  if (!dims_ok(M, N) || !valid_precision(precision)) return 0;
  return dict_bytes(M, N, precision);
}

int omp_dict_init(omp_dict_t *dict, const float *A, int64_t M, int64_t N, int64_t lda, int32_t precision,
                  void *mem, size_t bytes, void *stream) {
  if (!dict || !A || !dims_ok(M, N) || lda < M) return OMP_EINVAL;
  if (!valid_precision(precision)) return OMP_EINVAL;
  if (!aligned(A, 4)) return OMP_EINVAL;
  const size_t need = dict_bytes(M, N, precision);
  if (!mem || bytes < need || !aligned(mem, ALIGN)) return OMP_EWORKSPACE;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DictView d = dict_view(mem, M, N, precision);
  hipError_t e = launch_dict_prep(A, lda, d, st);
  if (e == hipSuccess) e = precision == OMP_PREC_FP64 ? launch_gram64(d, st) : launch_gram(d, st);
  if (e != hipSuccess) return device_error(e);
  dict->magic = DICT_MAGIC;
  dict->precision = precision;
  dict->M = M;
  dict->N = N;
  dict->Mp = d.Mp;
  dict->Np = d.Np;
  dict->A = A;
  dict->mem = mem;
  dict->bytes = bytes;
  return OMP_OK;
}

// Whether a solve runs in the Gram-domain form: on request (1), or automatically
// (2) for FP32 solves where it was measured faster than the residual-vector form
// (one MI355X, S = 32 with 2000 and 10,000 signals, S = 64 with 4096): every
// dictionary at most four times wider than long (4M >= N), tall ones included,
// except dictionaries under 1 MiB in FP32 in batches of more than 4096 signals,
// where the residual-vector form (its residual formed in the solve) is faster.
static bool gram_domain_form(int32_t mode, int prec, int64_t M, int64_t N, int64_t B) {
  if (mode == 1) return true;
  if (mode != 2 || prec != OMP_PREC_FP32) return false;
  return 4 * M >= N && (B <= 4096 || M * N * 4 >= ((int64_t)1 << 20));
}

size_t omp_workspace_size(int64_t M, int64_t N, int64_t B, int32_t S, const omp_opts_t *opts) {
  return solve_bytes(M, N, B, S, opts);
}

}  // extern "C"

size_t bomp::solve_bytes(int64_t M, int64_t N, int64_t B, int32_t S, const omp_opts_t *opts) {
  const int prec = opts ? opts->precision : OMP_PREC_FP32;
  if (!dims_ok(M, N) || B < 0 || B > ((int64_t)1 << 26) || S < 1 || S > OMP_MAX_S) return 0;
  if (!valid_precision(prec)) return 0;
  const int cfg = opts ? opts->tile_config : 0;
  if (cfg < 0 || cfg > MAX_TILE_CFG) return 0;
  const bool v0 = opts && opts->v0 == 1;
  size_t total = work_bytes(M, N, B, S, prec, cfg,
                            !v0 && opts && gram_domain_form(opts->gram_domain, prec, M, N, B),
                            opts && opts->flag_near_ties == 1, v0);
  if (!opts || !opts->dict) total += dict_bytes(M, N, prec);
  return total;
}

namespace bomp {

int solve_impl(const float *A, int64_t M, int64_t N, int64_t lda, const float *Y, int64_t B, int64_t ldy,
               int32_t S, float eps, float *X_out, int32_t *support_out, const omp_opts_t *opts, void *stream,
               void *workspace, size_t workspace_bytes, bool direct) {
  // ---- validation (host only) ----
  if (!opts) return OMP_EINVAL;
  const int prec = opts->precision;
  if (!valid_precision(prec)) return OMP_EINVAL;
  const int cfg = opts->tile_config;
  if (cfg < 0 || cfg > MAX_TILE_CFG) return OMP_EINVAL;
  if (opts->gram_on_the_fly != 0 && opts->gram_on_the_fly != 1) return OMP_EINVAL;
  if (opts->refactor != 0 && opts->refactor != 1) return OMP_EINVAL;
  if (opts->gram_domain < 0 || opts->gram_domain > 2) return OMP_EINVAL;
  if (opts->gram_domain == 1 && prec != OMP_PREC_FP32) return OMP_EINVAL;
  if (opts->flag_near_ties != 0 && opts->flag_near_ties != 1) return OMP_EINVAL;
  if (opts->v0 != 0 && opts->v0 != 1) return OMP_EINVAL;
  const bool f64 = prec == OMP_PREC_FP64;  // the FP64 form runs Algorithm v0 in FP64
  const bool v0 = opts->v0 == 1 || f64;
  if (v0 && (is_half(prec) || opts->gram_domain == 1 || opts->gram_on_the_fly || opts->refactor))
    return OMP_EINVAL;
  const bool gdom = !v0 && gram_domain_form(opts->gram_domain, prec, M, N, B);
  const bool ties = opts->flag_near_ties == 1;
  if (!dims_ok(M, N) || B < 0 || B > ((int64_t)1 << 26)) return OMP_EINVAL;
  if (S < 1 || S > M || S > N) return OMP_EINVAL;
  if (S > OMP_MAX_S) return OMP_ENOTSUPP;
  if (!solve_fits(M, N, B, S, prec, cfg)) return OMP_ENOTSUPP;
  if (std::isnan(eps)) return OMP_EINVAL;
  if (!A || lda < M || !aligned(A, 4)) return OMP_EINVAL;
  if (B > 0 && (!Y || ldy < M || !aligned(Y, 4) || !support_out)) return OMP_EINVAL;
  if (opts->dict) {
    const omp_dict_t *dd = opts->dict;
    if (dd->magic != DICT_MAGIC || dd->M != M || dd->N != N || dd->A != A || dd->precision != prec ||
        !dd->mem)
      return OMP_EINVAL;
  }
  const size_t wneed = work_bytes(M, N, B, S, prec, cfg, gdom, ties, v0);
  const size_t need = wneed + (opts->dict ? 0 : dict_bytes(M, N, prec));
  if (!workspace || workspace_bytes < need || !aligned(workspace, ALIGN)) return OMP_EWORKSPACE;
  if (B == 0) return OMP_OK;
  int rc = check_device();
  if (rc != OMP_OK) return rc;

  // ---- enqueue ----
  hipStream_t st = static_cast<hipStream_t>(stream);
  PhaseTimer timer(opts->phase_ms, opts->phase_launches, st);
  // Everything the solve launches, on stream `cs`, each launch through the timer.
  auto enqueue = [&](hipStream_t cs) -> hipError_t {
    DictView d;
    hipError_t e = hipSuccess;
    if (opts->dict) {
      d = dict_view(opts->dict->mem, M, N, prec);
    } else {
      void *dmem = static_cast<char *>(workspace) + wneed;
      d = dict_view(dmem, M, N, prec);
      e = timer.run(OMP_PHASE_DICT, [&] { return launch_dict_prep(A, lda, d, cs); });
      if (e == hipSuccess)
        e = timer.run(OMP_PHASE_DICT, [&] { return f64 ? launch_gram64(d, cs) : launch_gram(d, cs); });
      if (e != hipSuccess) return e;
    }
    WorkView w = work_view(workspace, M, N, B, S, prec, cfg, gdom, ties, v0);
    w.gram_fly = opts->gram_on_the_fly;
    w.refactor = opts->refactor;
    // the solve forms the residual itself where that was measured faster (one launch fewer per step)
    w.fuse_res = (!gdom && !v0 && !f64 && residual_in_solve(d, B)) ? 1 : 0;
    // the register-residual solve (512 < M <= 1024) forms it in a variant of its own, with one factor row per lane
    if (solve_rr(d, w) && S > 64) w.fuse_res = 0;
    e = timer.run(OMP_PHASE_INIT, [&] {
      return launch_init(Y, ldy, opts->S_per_signal, opts->eps_per_signal, eps, d, w, prec, cs);
    });
    if (f64) {
      // FP64 form: Algorithm v0 in FP64
      if (e == hipSuccess) e = timer.run(OMP_PHASE_INIT, [&] { return launch_project64(d, w, cs); });
      if (e == hipSuccess) e = timer.run(OMP_PHASE_INIT, [&] { return launch_v0_first64(d, w, cs); });
      for (int it = 0; it < S && e == hipSuccess; ++it)
        e = timer.run(OMP_PHASE_UPDATE, [&] { return launch_v0_step64(d, w, cs); });
      if (e == hipSuccess) e = timer.run(OMP_PHASE_OUTPUT, [&] { return launch_v0_coef64(w, cs); });
    } else if (v0) {
      // Algorithm v0: one kernel per step, the coefficients x = F u at the end
      if (e == hipSuccess) e = timer.run(OMP_PHASE_INIT, [&] { return launch_project(d, w, cs); });
      if (e == hipSuccess) e = timer.run(OMP_PHASE_INIT, [&] { return launch_v0_first(d, w, cs); });
      for (int it = 0; it < S && e == hipSuccess; ++it)
        e = timer.run(OMP_PHASE_UPDATE, [&] { return launch_v0_step(d, w, cs); });
      if (e == hipSuccess) e = timer.run(OMP_PHASE_OUTPUT, [&] { return launch_v0_coef(w, cs); });
    } else if (gdom && e == hipSuccess) {
      e = timer.run(OMP_PHASE_INIT, [&] { return launch_project(d, w, cs); });
    }
    for (int it = 0; it < S && e == hipSuccess && !v0; ++it) {
      if (gdom) {
        // Gram-domain form: correlations from P and G; no residual vectors
        e = timer.run(OMP_PHASE_CORR, [&] { return launch_gram_select(d, w, cs); });
        if (e == hipSuccess) e = timer.run(OMP_PHASE_UPDATE, [&] { return launch_solve(d, w, prec, cs); });
        continue;
      }
      e = timer.run(OMP_PHASE_CORR, [&] { return launch_corr_select(d, w, prec, cs); });
      if (e == hipSuccess) e = timer.run(OMP_PHASE_UPDATE, [&] { return launch_solve(d, w, prec, cs); });
      // after step it every signal holds at most it + 1 atoms
      if (e == hipSuccess && !w.fuse_res)
        e = timer.run(OMP_PHASE_RESIDUAL, [&] { return launch_residual(d, w, prec, it + 1, cs); });
    }
    if (e == hipSuccess)
      e = timer.run(OMP_PHASE_OUTPUT, [&] {
        return launch_finalize(d, w, X_out, support_out, opts->coef_out, opts->status_out, opts->rnorm_out, cs);
      });
    return e;
  };

  hipError_t e = hipSuccess;
  bool done = false;
  if (!direct && opts->use_graph && !timer.on()) {
    // The whole solve replayed from a hipGraph cached under every argument. On
    // the first use the launches are captured. (A timed call launches directly:
    // events recorded by graph nodes cannot be read back with elapsed times.)
    struct Key {
      const void *A, *Y, *X, *sup, *Sp, *Ep, *st_out, *rn_out, *coef, *dmem, *ws, *pool;
      int64_t M, N, lda, B, ldy;
      int32_t S, prec, cfg, gram_fly, refactor, gram_dom, ties, v0;
      uint32_t eps_bits, pad;
    } key;
    std::memset(&key, 0, sizeof(key));
    key.A = A;
    key.Y = Y;
    key.X = X_out;
    key.sup = support_out;
    key.Sp = opts->S_per_signal;
    key.Ep = opts->eps_per_signal;
    key.st_out = opts->status_out;
    key.rn_out = opts->rnorm_out;
    key.coef = opts->coef_out;
    key.dmem = opts->dict ? opts->dict->mem : nullptr;
    key.ws = workspace;
    key.pool = nullptr;
    key.M = M;
    key.N = N;
    key.lda = lda;
    key.B = B;
    key.ldy = ldy;
    key.S = S;
    key.prec = prec;
    key.cfg = cfg;
    key.gram_fly = opts->gram_on_the_fly;
    key.refactor = opts->refactor;
    key.gram_dom = gdom ? 1 : 0;
    key.ties = ties ? 1 : 0;
    key.v0 = v0 ? 1 : 0;
    std::memcpy(&key.eps_bits, &eps, sizeof(float));
    {
      const DictView dp = opts->dict ? dict_view(opts->dict->mem, M, N, prec)
                                     : dict_view(static_cast<char *>(workspace) + wneed, M, N, prec);
      e = prepare_kernels(dp, work_view(workspace, M, N, B, S, prec, cfg, gdom, ties, v0), prec, 0);
    }
    if (e == hipSuccess)
      e = graph_launch_cached(std::string(reinterpret_cast<const char *>(&key), sizeof(key)),
                              [&](hipStream_t cs) { return enqueue(cs); }, st);
    if (e == hipSuccess) {
      done = true;
    } else {
      (void)hipGetLastError();  // a failed capture falls back to direct launches
      e = hipSuccess;
    }
  }
  if (!done) {
    timer.reset();
    e = enqueue(st);
  }
  if (e == hipSuccess) e = timer.finish();
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

}  // namespace bomp

extern "C" {

int omp_solve(const float *A, int64_t M, int64_t N, int64_t lda, const float *Y, int64_t B, int64_t ldy,
              int32_t S, float eps, float *X_out, int32_t *support_out, const omp_opts_t *opts,
              void *stream) {
  if (!opts) return OMP_EINVAL;
  return solve_impl(A, M, N, lda, Y, B, ldy, S, eps, X_out, support_out, opts, stream, opts->workspace,
                    opts->workspace_bytes, false);
}

}  // extern "C"
