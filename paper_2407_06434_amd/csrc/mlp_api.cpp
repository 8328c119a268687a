// Host side of the learned support proposal: the network's memory layout,
// argument checks, and the sequences of kernels for features, forward pass,
// gradients, the Adam step and the learned solve with its OMP fallback.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/batched_omp.h"
#include "mlp_internal.h"
#include "omp_internal.h"

namespace bomp {
namespace {

constexpr uint32_t MLP_MAGIC = 0x4f4d4c50u;  // "OMLP"
constexpr int WSPLITS = 4;                   // split of the batch reduction in the weight gradients
constexpr int BCHUNKS = 16;                  // row chunks of the bias gradients
constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f, ADAM_EPS = 1e-8f;

size_t al(size_t x) { return (x + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = al(off);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

bool mlp_dims_ok(int64_t a, int64_t h, int64_t o) {
  return a >= 256 && h >= 256 && o >= 256 && a % 256 == 0 && h % 256 == 0 && o % 256 == 0 && a <= 16384 &&
         h <= 16384 && o <= 16384;
}

void layer_dims(int64_t ni, int64_t nh, int64_t no, int l, int64_t *in, int64_t *out) {
  *in = l == 0 ? ni : nh;
  *out = l == 2 ? no : nh;
}

// Network memory: per layer W32, W16, W16T, b32, mW, vW, mb, vb.
size_t mlp_layout(int64_t ni, int64_t nh, int64_t no, char *base, LayerView *L) {
  Carver c{base};
  for (int l = 0; l < 3; ++l) {
    int64_t in, out;
    layer_dims(ni, nh, no, l, &in, &out);
    LayerView v;
    v.n_in = in;
    v.n_out = out;
    v.W32 = c.take<float>(in * out);
    v.W16 = c.take<uint16_t>(in * out);
    v.W16T = c.take<uint16_t>(in * out);
    v.b32 = c.take<float>(out);
    v.mW = c.take<float>(in * out);
    v.vW = c.take<float>(in * out);
    v.mb = c.take<float>(out);
    v.vb = c.take<float>(out);
    if (L) L[l] = v;
  }
  return al(c.off);
}

bool mlp_ok(const omp_mlp_t *m) {
  return m && m->magic == MLP_MAGIC && m->mem && mlp_dims_ok(m->n_in, m->n_hidden, m->n_out);
}

// Training / inference buffers for a padded batch of Bp rows.
struct NetWork {
  int64_t Bp;
  uint16_t *F, *H1, *H2, *dZ, *dH2, *dH1;
  uint16_t *FT, *H1T, *H2T, *dZT, *dH2T, *dH1T;
  float *Z;
  uint32_t *labels;
  float *loss_part;
  float *gW[3], *gb[3];
  uint16_t *Y16;
  float *yinv;
  size_t total;
};

NetWork net_layout(int64_t ni, int64_t nh, int64_t no, int64_t M, int64_t B, char *base) {
  NetWork w;
  const int64_t Bp = round_up(std::max<int64_t>(B, 1), BPAD);
  const int64_t Mp = round_up(std::max<int64_t>(M, 1), KPAD);
  w.Bp = Bp;
  Carver c{base};
  w.F = c.take<uint16_t>(Bp * ni);
  w.H1 = c.take<uint16_t>(Bp * nh);
  w.H2 = c.take<uint16_t>(Bp * nh);
  w.dZ = c.take<uint16_t>(Bp * no);
  w.dH2 = c.take<uint16_t>(Bp * nh);
  w.dH1 = c.take<uint16_t>(Bp * nh);
  w.FT = c.take<uint16_t>(Bp * ni);
  w.H1T = c.take<uint16_t>(Bp * nh);
  w.H2T = c.take<uint16_t>(Bp * nh);
  w.dZT = c.take<uint16_t>(Bp * no);
  w.dH2T = c.take<uint16_t>(Bp * nh);
  w.dH1T = c.take<uint16_t>(Bp * nh);
  w.Z = c.take<float>(Bp * no);
  w.labels = c.take<uint32_t>(Bp * (no / 32));
  w.loss_part = c.take<float>(gemm_blocks(Bp, no, 1));
  for (int l = 0; l < 3; ++l) {
    int64_t in, out;
    layer_dims(ni, nh, no, l, &in, &out);
    w.gW[l] = c.take<float>((size_t)WSPLITS * in * out);
    w.gb[l] = c.take<float>((size_t)BCHUNKS * out);
  }
  w.Y16 = c.take<uint16_t>(Bp * Mp);
  w.yinv = c.take<float>(Bp);
  w.total = al(c.off);
  return w;
}

struct Net {
  LayerView L[3];
  int64_t ni, nh, no;
};

Net net_of(const omp_mlp_t *m) {
  Net n;
  n.ni = m->n_in;
  n.nh = m->n_hidden;
  n.no = m->n_out;
  mlp_layout(n.ni, n.nh, n.no, static_cast<char *>(m->mem), n.L);
  return n;
}

GemmEpi epi0() {
  GemmEpi e;
  std::memset(&e, 0, sizeof(e));
  return e;
}

// Forward pass on the padded batch w.F: H1, H2 and either FP32 scores (Z) or,
// when `labels` is given, the BCE output gradient dZ and the loss partials.
hipError_t forward(const Net &n, const NetWork &w, int64_t B, bool train, hipStream_t st) {
  const int64_t Bp = w.Bp;
  GemmEpi e = epi0();
  e.out = w.H1;
  e.ldo = n.nh;
  e.bias = n.L[0].b32;
  hipError_t err = launch_gemm_bf16(EPI_BIAS_RELU, w.F, n.ni, n.L[0].W16, n.ni, Bp, n.nh, n.ni, 1, e, st);
  if (err != hipSuccess) return err;
  e.out = w.H2;
  e.bias = n.L[1].b32;
  err = launch_gemm_bf16(EPI_BIAS_RELU, w.H1, n.nh, n.L[1].W16, n.nh, Bp, n.nh, n.nh, 1, e, st);
  if (err != hipSuccess) return err;
  e = epi0();
  e.bias = n.L[2].b32;
  e.ldo = n.no;
  if (!train) {
    e.out = w.Z;
    return launch_gemm_bf16(EPI_BIAS, w.H2, n.nh, n.L[2].W16, n.nh, Bp, n.no, n.nh, 1, e, st);
  }
  e.out = w.dZ;
  e.labels = w.labels;
  e.ldl = n.no / 32;
  e.mvalid = B;
  e.scale = 1.f / (float)B;
  e.loss_part = w.loss_part;
  return launch_gemm_bf16(EPI_BCE, w.H2, n.nh, n.L[2].W16, n.nh, Bp, n.no, n.nh, 1, e, st);
}

// Backward pass after forward(train): dH2, dH1, the activation transposes and
// the split partial sums of every gradient.
hipError_t backward(const Net &n, const NetWork &w, hipStream_t st) {
  const int64_t Bp = w.Bp;
  GemmEpi e = epi0();
  e.out = w.dH2;
  e.ldo = n.nh;
  e.mask = w.H2;
  hipError_t err = launch_gemm_bf16(EPI_RELU_MASK, w.dZ, n.no, n.L[2].W16T, n.no, Bp, n.nh, n.no, 1, e, st);
  if (err != hipSuccess) return err;
  e.out = w.dH1;
  e.mask = w.H1;
  err = launch_gemm_bf16(EPI_RELU_MASK, w.dH2, n.nh, n.L[1].W16T, n.nh, Bp, n.nh, n.nh, 1, e, st);
  if (err != hipSuccess) return err;
  const uint16_t *src[6] = {w.F, w.H1, w.H2, w.dZ, w.dH2, w.dH1};
  uint16_t *dst[6] = {w.FT, w.H1T, w.H2T, w.dZT, w.dH2T, w.dH1T};
  const int64_t cols[6] = {n.ni, n.nh, n.nh, n.no, n.nh, n.nh};
  for (int i = 0; i < 6 && err == hipSuccess; ++i) err = launch_transpose16(src[i], Bp, cols[i], dst[i], st);
  if (err != hipSuccess) return err;
  // dW_l[o][i] = sum_b dOut[b][o] In[b][i]; db_l[o] = sum_b dOut[b][o]
  const uint16_t *dOutT[3] = {w.dH1T, w.dH2T, w.dZT};
  const uint16_t *InT[3] = {w.FT, w.H1T, w.H2T};
  const uint16_t *dOut[3] = {w.dH1, w.dH2, w.dZ};
  for (int l = 0; l < 3 && err == hipSuccess; ++l) {
    GemmEpi g = epi0();
    g.out = w.gW[l];
    g.ldo = n.L[l].n_in;
    err = launch_gemm_bf16(EPI_PARTIAL, dOutT[l], Bp, InT[l], Bp, n.L[l].n_out, n.L[l].n_in, Bp, WSPLITS, g, st);
    if (err == hipSuccess) err = launch_colsum16(dOut[l], Bp, n.L[l].n_out, BCHUNKS, w.gb[l], st);
  }
  return err;
}

}  // namespace
}  // namespace bomp

using namespace bomp;

extern "C" {

size_t omp_mlp_size(int32_t n_in, int32_t n_hidden, int32_t n_out) {
  if (!mlp_dims_ok(n_in, n_hidden, n_out)) return 0;
  return mlp_layout(n_in, n_hidden, n_out, nullptr, nullptr);
}

int omp_mlp_init(omp_mlp_t *mlp, int32_t n_in, int32_t n_hidden, int32_t n_out, const float *const params[6],
                 void *mem, size_t bytes, void *stream) {
  if (!mlp || !params || !mlp_dims_ok(n_in, n_hidden, n_out)) return OMP_EINVAL;
  for (int i = 0; i < 6; ++i)
    if (!params[i] || !aligned(params[i], 4)) return OMP_EINVAL;
  if (!mem || bytes < mlp_layout(n_in, n_hidden, n_out, nullptr, nullptr) || !aligned(mem, WS_ALIGN))
    return OMP_EWORKSPACE;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  LayerView L[3];
  mlp_layout(n_in, n_hidden, n_out, static_cast<char *>(mem), L);
  hipError_t e = hipSuccess;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    const int64_t nw = L[l].n_in * L[l].n_out, nb = L[l].n_out;
    e = launch_copy32(params[2 * l], nw, L[l].W32, st);
    if (e == hipSuccess) e = launch_copy32(params[2 * l + 1], nb, L[l].b32, st);
    if (e == hipSuccess) e = launch_copy32(nullptr, nw, L[l].mW, st);
    if (e == hipSuccess) e = launch_copy32(nullptr, nw, L[l].vW, st);
    if (e == hipSuccess) e = launch_copy32(nullptr, nb, L[l].mb, st);
    if (e == hipSuccess) e = launch_copy32(nullptr, nb, L[l].vb, st);
    if (e == hipSuccess) e = launch_adam_w(L[l], nullptr, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0, st);  // BF16 copies
  }
  if (e != hipSuccess) return device_error(e);
  mlp->magic = MLP_MAGIC;
  mlp->n_in = n_in;
  mlp->n_hidden = n_hidden;
  mlp->n_out = n_out;
  mlp->step = 0;
  mlp->mem = mem;
  mlp->bytes = bytes;
  return OMP_OK;
}

int omp_mlp_export(const omp_mlp_t *mlp, float *const params[6], void *stream) {
  if (!mlp_ok(mlp) || !params) return OMP_EINVAL;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Net n = net_of(mlp);
  hipError_t e = hipSuccess;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    if (params[2 * l]) e = launch_copy32(n.L[l].W32, n.L[l].n_in * n.L[l].n_out, params[2 * l], st);
    if (e == hipSuccess && params[2 * l + 1]) e = launch_copy32(n.L[l].b32, n.L[l].n_out, params[2 * l + 1], st);
  }
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

size_t omp_mlp_workspace_size(const omp_mlp_t *mlp, int64_t M, int64_t B) {
  if (!mlp_ok(mlp) || B < 0 || B > ((int64_t)1 << 24) || M < 0 || M > ((int64_t)1 << 24)) return 0;
  return net_layout(mlp->n_in, mlp->n_hidden, mlp->n_out, M, B, nullptr).total;
}

int omp_mlp_features(const omp_dict_t *dict, const float *Y, int64_t B, int64_t ldy, uint16_t *F,
                     const omp_mlp_t *mlp, void *workspace, size_t workspace_bytes, void *stream) {
  if (!mlp_ok(mlp) || !dict || dict->magic != DICT_MAGIC || dict->precision != OMP_PREC_BF16 || !dict->mem)
    return OMP_EINVAL;
  if (dict->N != mlp->n_in || B < 0 || B > ((int64_t)1 << 24)) return OMP_EINVAL;
  if (B > 0 && (!Y || !F || ldy < dict->M || !aligned(Y, 4) || !aligned(F, 2))) return OMP_EINVAL;
  const size_t need = net_layout(mlp->n_in, mlp->n_hidden, mlp->n_out, dict->M, B, nullptr).total;
  if (!workspace || workspace_bytes < need || !aligned(workspace, WS_ALIGN)) return OMP_EWORKSPACE;
  if (B == 0) return OMP_OK;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const NetWork w = net_layout(mlp->n_in, mlp->n_hidden, mlp->n_out, dict->M, B, static_cast<char *>(workspace));
  const DictView d = dict_view(dict->mem, dict->M, dict->N, OMP_PREC_BF16);
  hipError_t e = launch_prep_signals(Y, ldy, B, d.M, d.Mp, w.Bp, w.Y16, w.yinv, st);
  GemmEpi g = epi0();
  g.out = w.F;
  g.ldo = d.Np;
  g.colscale = d.inv_nu;
  g.rowscale = w.yinv;
  g.scale = (float)std::sqrt((double)d.M);
  if (e == hipSuccess) e = launch_gemm_bf16(EPI_FEATURES, w.Y16, d.Mp, d.A16, d.Mp, w.Bp, d.Np, d.Mp, 1, g, st);
  if (e == hipSuccess) e = launch_pad_rows16(w.F, d.Np, nullptr, B, d.N, B, F, st);
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

int omp_mlp_forward(const omp_mlp_t *mlp, const uint16_t *F, int64_t B, float *Z, void *workspace,
                    size_t workspace_bytes, void *stream) {
  if (!mlp_ok(mlp) || B < 0 || B > ((int64_t)1 << 24)) return OMP_EINVAL;
  if (B > 0 && (!F || !Z || !aligned(F, 2) || !aligned(Z, 4))) return OMP_EINVAL;
  const size_t need = net_layout(mlp->n_in, mlp->n_hidden, mlp->n_out, 0, B, nullptr).total;
  if (!workspace || workspace_bytes < need || !aligned(workspace, WS_ALIGN)) return OMP_EWORKSPACE;
  if (B == 0) return OMP_OK;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Net n = net_of(mlp);
  const NetWork w = net_layout(n.ni, n.nh, n.no, 0, B, static_cast<char *>(workspace));
  hipError_t e = launch_pad_rows16(F, n.ni, nullptr, B, n.ni, w.Bp, w.F, st);
  if (e == hipSuccess) e = forward(n, w, B, false, st);
  if (e == hipSuccess) e = launch_copy32(w.Z, B * n.no, Z, st);
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

static int grad_common(const omp_mlp_t *mlp, const uint16_t *F, const int32_t *support, const int32_t *rows,
                       int64_t B, int32_t S,
                       float *loss_out, void *workspace, size_t workspace_bytes, hipStream_t st, Net *net,
                       NetWork *nw) {
  if (!mlp_ok(mlp) || B < 1 || B > ((int64_t)1 << 24) || S < 1 || S > mlp->n_out) return OMP_EINVAL;
  if (!F || !support || !aligned(F, 2) || !aligned(support, 4) || !aligned(rows, 4)) return OMP_EINVAL;
  const size_t need = net_layout(mlp->n_in, mlp->n_hidden, mlp->n_out, 0, B, nullptr).total;
  if (!workspace || workspace_bytes < need || !aligned(workspace, WS_ALIGN)) return OMP_EWORKSPACE;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  *net = net_of(mlp);
  const Net &n = *net;
  *nw = net_layout(n.ni, n.nh, n.no, 0, B, static_cast<char *>(workspace));
  const NetWork &w = *nw;
  hipError_t e = launch_pad_rows16(F, n.ni, rows, B, n.ni, w.Bp, w.F, st);
  if (e == hipSuccess) e = launch_labels(support, rows, B, S, n.no, w.Bp, w.labels, st);
  if (e == hipSuccess) e = forward(n, w, B, true, st);
  if (e == hipSuccess && loss_out)
    e = launch_loss_sum(w.loss_part, gemm_blocks(w.Bp, n.no, 1), 1.f / (float)B, loss_out, st);
  if (e == hipSuccess) e = backward(n, w, st);
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

int omp_mlp_grad(const omp_mlp_t *mlp, const uint16_t *F, const int32_t *support, const int32_t *rows, int64_t B,
                 int32_t S, float *loss_out, float *const grads_out[6], void *workspace, size_t workspace_bytes,
                 void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  Net n;
  NetWork w;
  int rc = grad_common(mlp, F, support, rows, B, S, loss_out, workspace, workspace_bytes, st, &n, &w);
  if (rc != OMP_OK || !grads_out) return rc;
  hipError_t e = hipSuccess;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    if (grads_out[2 * l])
      e = launch_sum_parts(w.gW[l], WSPLITS, n.L[l].n_in * n.L[l].n_out, grads_out[2 * l], st);
    if (e == hipSuccess && grads_out[2 * l + 1])
      e = launch_sum_parts(w.gb[l], BCHUNKS, n.L[l].n_out, grads_out[2 * l + 1], st);
  }
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

int omp_mlp_train_step(omp_mlp_t *mlp, const uint16_t *F, const int32_t *support, const int32_t *rows, int64_t B,
                       int32_t S, float lr, float *loss_out, void *workspace, size_t workspace_bytes, void *stream) {
  if (!(lr >= 0.f) || !std::isfinite(lr)) return OMP_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Net n;
  NetWork w;
  int rc = grad_common(mlp, F, support, rows, B, S, loss_out, workspace, workspace_bytes, st, &n, &w);
  if (rc != OMP_OK) return rc;
  const int64_t t = mlp->step + 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)ADAM_B1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)ADAM_B2, (double)t)));
  hipError_t e = hipSuccess;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    e = launch_adam_w(n.L[l], w.gW[l], WSPLITS, lr, ADAM_B1, ADAM_B2, ADAM_EPS, c1, c2, 1, st);
    if (e == hipSuccess) e = launch_adam_b(n.L[l], w.gb[l], BCHUNKS, lr, ADAM_B1, ADAM_B2, ADAM_EPS, c1, c2, st);
  }
  if (e != hipSuccess) return device_error(e);
  mlp->step = t;
  return OMP_OK;
}

// ---- learned solve ----------------------------------------------------------

namespace {
struct SolveLayout {
  NetWork net;
  size_t off_P, off_acc, off_idx, off_cnt, off_Yr, off_epsr, off_sup, off_coef, off_st, off_rn, off_omp, total;
};

SolveLayout solve_layout(const omp_dict_t *dict, const omp_mlp_t *mlp, int64_t B, int32_t S, int cfg) {
  SolveLayout L;
  L.net = net_layout(mlp->n_in, mlp->n_hidden, mlp->n_out, dict->M, B, nullptr);
  const int64_t Bp = L.net.Bp;
  size_t off = L.net.total;
  auto take = [&](size_t bytes) {
    off = al(off);
    const size_t at = off;
    off += bytes;
    return at;
  };
  L.off_P = take((size_t)Bp * S * 4);
  L.off_acc = take((size_t)Bp * 4);
  L.off_idx = take((size_t)Bp * 4);
  L.off_cnt = take(4);
  L.off_Yr = take((size_t)Bp * dict->M * 4);
  L.off_epsr = take((size_t)Bp * 4);
  L.off_sup = take((size_t)Bp * S * 4);
  L.off_coef = take((size_t)Bp * S * 4);
  L.off_st = take((size_t)Bp * 4);
  L.off_rn = take((size_t)Bp * 4);
  omp_opts_t o;
  omp_opts_default(&o);
  o.precision = dict->precision;
  o.tile_config = cfg;
  o.dict = dict;
  L.off_omp = take(omp_workspace_size(dict->M, dict->N, B, S, &o));
  L.total = al(off);
  return L;
}
}  // namespace

size_t omp_learned_workspace_size(const omp_dict_t *dict, const omp_mlp_t *mlp, int64_t B, int32_t S,
                                  const omp_opts_t *fallback) {
  if (!mlp_ok(mlp) || !dict || dict->magic != DICT_MAGIC || dict->precision != OMP_PREC_BF16) return 0;
  if (dict->N != mlp->n_in || dict->N != mlp->n_out || B < 0 || B > ((int64_t)1 << 24)) return 0;
  if (S < 1 || S > 64 || S > dict->M || S > dict->N) return 0;
  const int cfg = fallback ? fallback->tile_config : 0;
  if (cfg < 0 || cfg > MAX_TILE_CFG) return 0;
  return solve_layout(dict, mlp, B, S, cfg).total;
}

int omp_learned_solve(const omp_dict_t *dict, const omp_mlp_t *mlp, const float *Y, int64_t B, int64_t ldy,
                      int32_t S, float eps, const float *eps_per_signal, int32_t *support_out, float *coef_out,
                      int32_t *status_out, float *rnorm_out, int64_t *accepted_out, const omp_opts_t *fallback,
                      void *workspace, size_t workspace_bytes, void *stream) {
  if (!mlp_ok(mlp) || !dict || dict->magic != DICT_MAGIC || dict->precision != OMP_PREC_BF16 || !dict->mem)
    return OMP_EINVAL;
  if (dict->N != mlp->n_in || dict->N != mlp->n_out || B < 0 || B > ((int64_t)1 << 24)) return OMP_EINVAL;
  if (S < 1 || S > dict->M || S > dict->N) return OMP_EINVAL;
  if (S > 64) return OMP_ENOTSUPP;
  if (std::isnan(eps)) return OMP_EINVAL;
  const int cfg = fallback ? fallback->tile_config : 0;
  if (cfg < 0 || cfg > MAX_TILE_CFG) return OMP_EINVAL;
  if (B > 0 && (!Y || ldy < dict->M || !aligned(Y, 4) || !support_out || !coef_out || !status_out || !rnorm_out))
    return OMP_EINVAL;
  const SolveLayout L = solve_layout(dict, mlp, B, S, cfg);
  if (!workspace || workspace_bytes < L.total || !aligned(workspace, WS_ALIGN)) return OMP_EWORKSPACE;
  if (accepted_out) *accepted_out = 0;
  if (B == 0) return OMP_OK;
  int rc = check_device();
  if (rc != OMP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *ws = static_cast<char *>(workspace);
  const Net n = net_of(mlp);
  const NetWork w = net_layout(n.ni, n.nh, n.no, dict->M, B, ws);
  const DictView d = dict_view(dict->mem, dict->M, dict->N, OMP_PREC_BF16);
  int32_t *P = reinterpret_cast<int32_t *>(ws + L.off_P);
  int32_t *acc = reinterpret_cast<int32_t *>(ws + L.off_acc);
  int32_t *idx = reinterpret_cast<int32_t *>(ws + L.off_idx);
  int32_t *cnt = reinterpret_cast<int32_t *>(ws + L.off_cnt);
  float *Yr = reinterpret_cast<float *>(ws + L.off_Yr);
  float *epsr = reinterpret_cast<float *>(ws + L.off_epsr);
  int32_t *sup_r = reinterpret_cast<int32_t *>(ws + L.off_sup);
  float *coef_r = reinterpret_cast<float *>(ws + L.off_coef);
  int32_t *st_r = reinterpret_cast<int32_t *>(ws + L.off_st);
  float *rn_r = reinterpret_cast<float *>(ws + L.off_rn);

  // features -> network -> proposal -> check -> compaction of the rejects
  hipError_t e = launch_prep_signals(Y, ldy, B, d.M, d.Mp, w.Bp, w.Y16, w.yinv, st);
  GemmEpi g = epi0();
  g.out = w.F;
  g.ldo = d.Np;
  g.colscale = d.inv_nu;
  g.rowscale = w.yinv;
  g.scale = (float)std::sqrt((double)d.M);
  if (e == hipSuccess) e = launch_gemm_bf16(EPI_FEATURES, w.Y16, d.Mp, d.A16, d.Mp, w.Bp, d.Np, d.Mp, 1, g, st);
  if (e == hipSuccess) e = forward(n, w, B, false, st);
  if (e == hipSuccess) e = launch_topk(w.Z, n.no, n.no, B, S, P, st);
  if (e == hipSuccess)
    e = launch_ls_check(d, Y, ldy, B, P, S, eps_per_signal, eps, support_out, coef_out, status_out, rnorm_out, acc,
                        st);
  if (e == hipSuccess) e = launch_compact(acc, B, idx, cnt, st);
  int32_t nrej = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nrej, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return device_error(e);
  if (accepted_out) *accepted_out = B - nrej;
  if (nrej == 0) return OMP_OK;

  // fallback: plain OMP on the rejected signals, results scattered back
  e = launch_gather_rejects(Y, ldy, d.M, eps_per_signal, eps, idx, nrej, Yr, epsr, st);
  if (e != hipSuccess) return device_error(e);
  omp_opts_t o;
  omp_opts_default(&o);
  o.precision = dict->precision;
  o.tile_config = cfg;
  o.dict = dict;
  o.eps_per_signal = epsr;
  o.status_out = st_r;
  o.rnorm_out = rn_r;
  o.coef_out = coef_r;
  o.workspace = ws + L.off_omp;
  o.workspace_bytes = workspace_bytes - L.off_omp;
  rc = omp_solve(dict->A, d.M, d.N, d.M, Yr, nrej, d.M, S, eps, nullptr, sup_r, &o, stream);
  if (rc != OMP_OK) return rc;
  e = launch_scatter_fallback(idx, nrej, S, sup_r, coef_r, st_r, rn_r, support_out, coef_out, status_out, rnorm_out,
                              st);
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

}  // extern "C"
