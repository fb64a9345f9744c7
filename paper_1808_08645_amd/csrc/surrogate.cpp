// Host side of the trace surrogate (include/bbwadg_surrogate.h): layer table, parameter
// initialisation, buffers, and the forward, backward and Adam passes as sequences of the
// kernels in surrogate_kernel.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bbwadg.h"
#include "../../include/bbwadg_surrogate.h"
#include "surrogate_internal.hpp"

using namespace bbw;

namespace {

struct Layer {
  bool conv = false;
  int Cin = 0, Cout = 0, D = 0, Do = 0;  // convolution: D^3 x Cin -> Do^3 x Cout
  int64_t K = 0, Kp = 0, N = 0;          // GEMM inner size (padded) and output width
  bool relu = true;
  int64_t woff = 0, boff = 0;
  int64_t rows(int B) const { return conv ? (int64_t)B * Do * Do * Do : B; }
};

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int hipc(hipError_t e, const char* what) {
  return e == hipSuccess ? 0 : set_error(BBWADG_EHIP, "%s: %s", what, hipGetErrorString(e));
}
int kc(int e, const char* what) {
  return e == 0 ? 0 : set_error(BBWADG_EHIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

}  // namespace

struct bbwadg_sur {
  int grid = 16, nout = 0, max_batch = 0;
  std::vector<Layer> L;
  int64_t nparam = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* wbf = nullptr;
  uint16_t* xbf = nullptr;
  std::vector<float*> act, dy, dcol;    // per layer
  std::vector<uint16_t*> actbf, col;    // per layer
  uint16_t* dybf = nullptr;
  float* part = nullptr;        // split-K partial sums
  int64_t part_size = 0;
  double* partial = nullptr;
  int nred = 256;
  int64_t step = 0;
  std::vector<void*> owned;

  int alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) return set_error(BBWADG_ENOMEM, "device allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
    owned.push_back(*p);
    return 0;
  }
  ~bbwadg_sur() {
    if (!owned.empty()) (void)hipDeviceSynchronize();
    for (void* p : owned) (void)hipFree(p);
  }
};

namespace {

// Split K when the output has few 64 x 64 blocks and K is long: at most kMaxSplit slices of
// at least 256, into the context's partial-sum scratch.
constexpr int kMaxSplit = 64;

void choose_split(bbwadg_sur* s, GemmArgs& g) {
  const int64_t blocks = ((g.M + 63) / 64) * ((g.N + 63) / 64);
  int64_t S = 1;
  if (blocks < 128 && g.K >= 512) S = std::min<int64_t>({kMaxSplit, g.K / 256, (512 + blocks - 1) / blocks});
  while (S > 1 && S * g.M * g.N > s->part_size) --S;
  if (S > 1) {
    g.ksplit = (int32_t)S;
    g.kc = ((g.K + S - 1) / S + 15) / 16 * 16;
    g.ksplit = (int32_t)((g.K + g.kc - 1) / g.kc);
    g.part = s->part;
  }
}

int forward(bbwadg_sur* s, const float* x, int B, hipStream_t st) {
  int rc;
  const int64_t nin = (int64_t)B * s->grid * s->grid * s->grid;
  if ((rc = kc(sur_cast_bf16(x, s->xbf, nin, st), "cast"))) return rc;
  const uint16_t* in = s->xbf;
  for (size_t l = 0; l < s->L.size(); ++l) {
    const Layer& y = s->L[l];
    GemmArgs g{};
    if (y.conv) {
      if ((rc = kc(sur_im2col(in, s->col[l], B, y.D, y.Cin, y.Do, (int)y.Kp, st), "im2col"))) return rc;
      g.A = s->col[l];
    } else {
      g.A = in;
    }
    g.B = s->wbf + y.woff;
    g.C = s->act[l];
    g.Cbf = l + 1 < s->L.size() ? s->actbf[l] : nullptr;
    g.bias = s->w + y.boff;
    g.M = y.rows(B);
    g.N = y.N;
    g.K = y.Kp;
    g.sam = y.Kp;
    g.sak = 1;
    g.sbk = y.N;
    g.sbn = 1;
    g.ldc = y.N;
    g.relu = y.relu;
    choose_split(s, g);
    if ((rc = kc(sur_gemm(g, st), "gemm"))) return rc;
    in = s->actbf[l];
  }
  return 0;
}

// Gradient of the loss with respect to every parameter, from dL/dy in s->dy.back(); with
// dx0 != null also with respect to the input, into dx0 [B][grid^3].
int backward(bbwadg_sur* s, int B, hipStream_t st, float* dx0 = nullptr) {
  int rc;
  for (int l = (int)s->L.size() - 1; l >= 0; --l) {
    const Layer& y = s->L[l];
    const int64_t rows = y.rows(B);
    float* dy = s->dy[l];
    if (y.relu && (rc = kc(sur_relu_bwd(dy, s->act[l], rows * y.N, st), "relu"))) return rc;
    if ((rc = kc(sur_cast_bf16(dy, s->dybf, rows * y.N, st), "cast")) ||
        (rc = kc(sur_colsum(dy, s->g + y.boff, rows, y.N, st), "colsum")))
      return rc;
    // dW = X^T dY, X the layer's GEMM input [rows][Kp]
    GemmArgs g{};
    g.A = y.conv ? s->col[l] : (l > 0 ? s->actbf[l - 1] : s->xbf);
    g.sam = 1;
    g.sak = y.Kp;
    g.B = s->dybf;
    g.sbk = y.N;
    g.sbn = 1;
    g.C = s->g + y.woff;
    g.ldc = y.N;
    g.M = y.Kp;
    g.N = y.N;
    g.K = rows;
    choose_split(s, g);
    if ((rc = kc(sur_gemm(g, st), "gemm dW"))) return rc;
    if (l == 0 && !dx0) break;
    // dX = dY W^T: into the previous layer's output gradient (through col2im for a convolution),
    // or for the first layer into the input gradient
    GemmArgs h{};
    h.A = s->dybf;
    h.sam = y.N;
    h.sak = 1;
    h.B = s->wbf + y.woff;
    h.sbk = 1;
    h.sbn = y.N;
    h.M = rows;
    h.N = y.Kp;
    h.K = y.N;
    h.C = y.conv ? s->dcol[l] : s->dy[l - 1];
    h.ldc = y.Kp;
    choose_split(s, h);
    if ((rc = kc(sur_gemm(h, st), "gemm dX"))) return rc;
    if (y.conv && (rc = kc(sur_col2im(s->dcol[l], l > 0 ? s->dy[l - 1] : dx0, B, y.D, y.Cin, y.Do, (int)y.Kp, st),
                           "col2im")))
      return rc;
  }
  return 0;
}

int loss_grad(bbwadg_sur* s, const float* x, const float* t, int B, double* loss, hipStream_t st,
              float* dx = nullptr) {
  int rc;
  if ((rc = forward(s, x, B, st))) return rc;
  const int64_t n = (int64_t)B * s->nout;
  if ((rc = kc(sur_mse(s->act.back(), t, s->dy.back(), s->partial, n, s->nred, st), "mse")) ||
      (rc = backward(s, B, st, dx)))
    return rc;
  std::vector<double> part(s->nred);
  if ((rc = hipc(hipMemcpyAsync(part.data(), s->partial, s->nred * 8, hipMemcpyDeviceToHost, st), "loss download")) ||
      (rc = hipc(hipStreamSynchronize(st), "sync")))
    return rc;
  double sum = 0;
  for (double p : part) sum += p;
  *loss = sum / (double)n;
  return 0;
}

int check_batch(const bbwadg_sur* s, int B) {
  return (B < 1 || B > s->max_batch) ? set_error(BBWADG_EINVAL, "batch %d outside [1, %d]", B, s->max_batch) : 0;
}

}  // namespace

extern "C" {

int bbwadg_sur_create(int32_t grid, int32_t nout, int32_t max_batch, uint64_t seed, bbwadg_sur** out) {
  if (!out) return set_error(BBWADG_EINVAL, "NULL output");
  *out = nullptr;
  if (grid != 16) return set_error(BBWADG_EINVAL, "grid must be 16");
  if (nout < 1 || nout > (1 << 24)) return set_error(BBWADG_EINVAL, "nout %d out of range", nout);
  if (max_batch < 1 || max_batch > 4096) return set_error(BBWADG_EINVAL, "max_batch %d outside [1, 4096]", max_batch);
  bbwadg_sur* s = new (std::nothrow) bbwadg_sur();
  if (!s) return set_error(BBWADG_ENOMEM, "surrogate");
  s->grid = grid;
  s->nout = nout;
  s->max_batch = max_batch;
  // layer table
  const int chans[4] = {1, 16, 32, 64};
  int D = grid;
  for (int i = 0; i < 3; ++i) {
    Layer y;
    y.conv = true;
    y.Cin = chans[i];
    y.Cout = chans[i + 1];
    y.D = D;
    y.Do = D / 2;
    y.K = 27 * y.Cin;
    y.Kp = (y.K + 15) / 16 * 16;
    y.N = y.Cout;
    s->L.push_back(y);
    D /= 2;
  }
  const int64_t dense[5] = {64 * 8, 256, 256, 64, nout};
  for (int i = 0; i < 4; ++i) {
    Layer y;
    y.Cin = (int)dense[i];
    y.Cout = (int)dense[i + 1];
    y.K = y.Kp = dense[i];
    y.N = dense[i + 1];
    y.relu = i < 3;
    s->L.push_back(y);
  }
  int64_t off = 0;
  for (Layer& y : s->L) {
    y.woff = off;
    off += y.Kp * y.N;
    y.boff = off;
    off += y.N;
  }
  s->nparam = off;
  // parameters
  std::vector<float> w((size_t)off, 0.f);
  for (const Layer& y : s->L) {
    const double a = std::sqrt((y.relu ? 6.0 : 3.0) / (double)y.K);
    for (int64_t k = 0; k < y.K; ++k)
      for (int64_t n = 0; n < y.N; ++n) {
        const int64_t i = y.woff + k * y.N + n;
        const double u = (double)(splitmix64(seed ^ splitmix64((uint64_t)i)) >> 11) * (1.0 / 9007199254740992.0);
        w[(size_t)i] = (float)((2.0 * u - 1.0) * a);
      }
  }
  int rc = 0;
  const size_t np = (size_t)off;
  if ((rc = s->alloc((void**)&s->w, np * 4)) || (rc = s->alloc((void**)&s->g, np * 4)) ||
      (rc = s->alloc((void**)&s->m, np * 4)) || (rc = s->alloc((void**)&s->v, np * 4)) ||
      (rc = s->alloc((void**)&s->wbf, np * 2)) ||
      (rc = s->alloc((void**)&s->xbf, (size_t)max_batch * grid * grid * grid * 2)) ||
      (rc = s->alloc((void**)&s->partial, (size_t)s->nred * 8))) {
    delete s;
    return rc;
  }
  size_t maxdy = 0;
  for (size_t l = 0; l < s->L.size(); ++l) {
    const Layer& y = s->L[l];
    const size_t n = (size_t)y.rows(max_batch) * y.N;
    float *a = nullptr, *d = nullptr, *dc = nullptr;
    uint16_t *ab = nullptr, *cl = nullptr;
    if ((rc = s->alloc((void**)&a, n * 4)) || (rc = s->alloc((void**)&ab, n * 2)) || (rc = s->alloc((void**)&d, n * 4)) ||
        (y.conv && ((rc = s->alloc((void**)&cl, (size_t)y.rows(max_batch) * y.Kp * 2)) ||
                    (rc = s->alloc((void**)&dc, (size_t)y.rows(max_batch) * y.Kp * 4))))) {
      delete s;
      return rc;
    }
    s->act.push_back(a);
    s->actbf.push_back(ab);
    s->dy.push_back(d);
    s->col.push_back(cl);
    s->dcol.push_back(dc);
    maxdy = std::max(maxdy, n);
  }
  s->part_size = (int64_t)1 << 22;  // 16 MB of partial sums
  if ((rc = s->alloc((void**)&s->dybf, maxdy * 2)) || (rc = s->alloc((void**)&s->part, (size_t)s->part_size * 4)) ||
      (rc = bbwadg_sur_set_params(s, w.data()))) {
    delete s;
    return rc;
  }
  *out = s;
  return 0;
}

int bbwadg_sur_destroy(bbwadg_sur* s) {
  delete s;
  return 0;
}

int64_t bbwadg_sur_num_params(const bbwadg_sur* s) { return s ? s->nparam : set_error(BBWADG_EINVAL, "NULL surrogate"); }

int bbwadg_sur_layout(const bbwadg_sur* s, int32_t layer, int32_t* info) {
  if (!s || !info) return set_error(BBWADG_EINVAL, "NULL argument");
  if (layer < 0 || layer >= (int)s->L.size()) return set_error(BBWADG_EINVAL, "layer %d outside [0, %zu)", layer, s->L.size());
  const Layer& y = s->L[layer];
  const int32_t v[8] = {y.conv, y.Cin, y.Cout, (int32_t)y.K, (int32_t)y.Kp, y.relu, (int32_t)y.woff, (int32_t)y.boff};
  std::memcpy(info, v, sizeof v);
  return 0;
}

int bbwadg_sur_get_params(const bbwadg_sur* s, float* host) {
  if (!s || !host) return set_error(BBWADG_EINVAL, "NULL argument");
  return hipc(hipMemcpy(host, s->w, (size_t)s->nparam * 4, hipMemcpyDeviceToHost), "parameter download");
}

int bbwadg_sur_set_params(bbwadg_sur* s, const float* host) {
  if (!s || !host) return set_error(BBWADG_EINVAL, "NULL argument");
  for (int64_t i = 0; i < s->nparam; ++i)
    if (!std::isfinite(host[i])) return set_error(BBWADG_EINVAL, "parameter %lld not finite", (long long)i);
  const size_t np = (size_t)s->nparam;
  int rc;
  if ((rc = hipc(hipMemcpy(s->w, host, np * 4, hipMemcpyHostToDevice), "parameter upload")) ||
      (rc = hipc(hipMemset(s->m, 0, np * 4), "memset")) || (rc = hipc(hipMemset(s->v, 0, np * 4), "memset")) ||
      (rc = hipc(hipMemset(s->g, 0, np * 4), "memset")) || (rc = kc(sur_cast_bf16(s->w, s->wbf, s->nparam, nullptr), "cast")) ||
      (rc = hipc(hipDeviceSynchronize(), "sync")))
    return rc;
  s->step = 0;
  return 0;
}

int bbwadg_sur_forward(bbwadg_sur* s, const float* x, int32_t B, float* y, void* stream) {
  if (!s || !x || !y) return set_error(BBWADG_EINVAL, "NULL argument");
  int rc = check_batch(s, B);
  hipStream_t st = (hipStream_t)stream;
  if (rc || (rc = forward(s, x, B, st))) return rc;
  return hipc(hipMemcpyAsync(y, s->act.back(), (size_t)B * s->nout * 4, hipMemcpyDeviceToDevice, st), "output copy");
}

int bbwadg_sur_loss_grad(bbwadg_sur* s, const float* x, const float* t, int32_t B, double* loss, float* grad_host,
                         void* stream) {
  if (!s || !x || !t || !loss) return set_error(BBWADG_EINVAL, "NULL argument");
  int rc = check_batch(s, B);
  hipStream_t st = (hipStream_t)stream;
  if (rc || (rc = loss_grad(s, x, t, B, loss, st))) return rc;
  if (grad_host)
    return hipc(hipMemcpy(grad_host, s->g, (size_t)s->nparam * 4, hipMemcpyDeviceToHost), "gradient download");
  return 0;
}

int bbwadg_sur_input_grad(bbwadg_sur* s, const float* x, const float* t, int32_t B, double* loss, float* dx,
                          void* stream) {
  if (!s || !x || !t || !loss || !dx) return set_error(BBWADG_EINVAL, "NULL argument");
  int rc = check_batch(s, B);
  hipStream_t st = (hipStream_t)stream;
  if (rc || (rc = loss_grad(s, x, t, B, loss, st, dx))) return rc;
  return 0;
}

int bbwadg_sur_train_step(bbwadg_sur* s, const float* x, const float* t, int32_t B, float lr, double* loss, void* stream) {
  if (!s || !x || !t || !loss) return set_error(BBWADG_EINVAL, "NULL argument");
  if (!(lr > 0.f) || !std::isfinite(lr)) return set_error(BBWADG_EINVAL, "learning rate must be finite and positive");
  int rc = check_batch(s, B);
  hipStream_t st = (hipStream_t)stream;
  if (rc || (rc = loss_grad(s, x, t, B, loss, st))) return rc;
  s->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)s->step)), c2 = (float)(1.0 - std::pow(0.999, (double)s->step));
  return kc(sur_adam(s->w, s->g, s->m, s->v, s->wbf, s->nparam, lr, b1, b2, 1e-8f, c1, c2, st), "adam");
}

}  // extern "C"
