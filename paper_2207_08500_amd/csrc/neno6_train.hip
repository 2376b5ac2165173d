// Classifier training (Sec. 3.3): binary cross entropy averaged over the
// four outputs and the mini-batch (eq. Crossentropy), hand-written backward
// pass, Adam.
//
// Gradient kernel: a block takes a tile of samples; each lane runs one sample
// forward (activations in registers, never written to memory) and backward,
// then the block reduces the per-sample outer products delta_l h_{l-1}^T
// through LDS in a fixed order and writes one partial gradient per block.
// A second kernel sums the partials over blocks in block order (FP64) and
// applies the Adam step, so results do not depend on scheduling.
#include "neno6_device.h"
#include "neno6_fast.h"

namespace n6 {

namespace {

constexpr int TB = 64;  // samples per block (one wave)

N6_DEV const float *uniform_f(const float *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const float *)(((uint64_t)hi << 32) | lo);
}

N6_DEV float softplus(float x) { return x > 0.f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }
N6_DEV float sigmoid(float x) { return 1.f / (1.f + expf(-x)); }

// Block reduction of sum_s d[s][o] * h[s][i] (o < NO, i < NI) and of
// sum_s d[s][o] into gW (row-major [o][i]) and gb.  d and h live in LDS as
// [s][.] for the TB samples of the block.
template <int NO, int NI>
N6_DEV void outer_reduce(const float *d, const float *h, int nvalid, float *gW, float *gb) {
  for (int e = threadIdx.x; e < NO * NI + NO; e += TB) {
    float acc = 0.f;
    if (e < NO * NI) {
      const int o = e / NI, i = e % NI;
      for (int s = 0; s < nvalid; ++s) acc = fmaf(d[s * NO + o], h[s * NI + i], acc);
      gW[e] = acc;
    } else {
      const int o = e - NO * NI;
      for (int s = 0; s < nvalid; ++s) acc += d[s * NO + o];
      gb[o] = acc;
    }
  }
}

// One block: samples idx[blockIdx.x * TB + t]; writes its partial gradient
// part[blockIdx.x][3228] and partial loss lpart[blockIdx.x] (FP32 sums).
__global__ void __launch_bounds__(TB)
k_grad_f32(const float *__restrict__ P32, const float *__restrict__ s, const uint8_t *__restrict__ y,
           const int64_t *__restrict__ idx, int64_t m, float inv_scale, float *__restrict__ part,
           double *__restrict__ lpart) {
  __shared__ float dl[TB * 64];
  __shared__ float hl[TB * 64];
  __shared__ float lsum[TB];
  const float *P = uniform_f(P32);
  const int64_t sample = blockIdx.x * (int64_t)TB + threadIdx.x;
  const bool valid = sample < m;
  const int nvalid = (int)((m - blockIdx.x * (int64_t)TB) < TB ? (m - blockIdx.x * (int64_t)TB) : TB);
  float x0[6] = {0, 0, 0, 0, 0, 0};
  unsigned lab = 0;
  if (valid) {
    const int64_t id = idx ? idx[sample] : sample;
    float st[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) st[j] = s[6 * id + j];
    features<float>(st, x0);
    lab = y[id];
  }
  // forward, activations kept in registers
  float h1[64], h2[32], h3[16], h4[8], z[4];
  dense<float, 6, 64, true>(P + OW1, P + OB1, x0, h1);
  dense<float, 64, 32, true>(P + OW2, P + OB2, h1, h2);
  dense<float, 32, 16, true>(P + OW3, P + OB3, h2, h3);
  dense<float, 16, 8, true>(P + OW4, P + OB4, h3, h4);
  dense<float, 8, 4, false>(P + OW5, P + OB5, h4, z);
  float loss = 0.f, d5[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float yk = (float)((lab >> k) & 1u);
    loss += yk * softplus(-z[k]) + (1.f - yk) * softplus(z[k]);
    d5[k] = valid ? (sigmoid(z[k]) - yk) * 0.25f * inv_scale : 0.f;
  }
  lsum[threadIdx.x] = valid ? 0.25f * loss : 0.f;
  // backward: delta_{l-1} = W_l^T delta_l masked by the ReLU of layer l-1
  float d4[8], d3[16], d2[32], d1[64];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float a = 0.f;
#pragma unroll
    for (int o = 0; o < 4; ++o) a = fmaf(P[OW5 + o * 8 + i], d5[o], a);
    d4[i] = h4[i] > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    float a = 0.f;
#pragma unroll
    for (int o = 0; o < 8; ++o) a = fmaf(P[OW4 + o * 16 + i], d4[o], a);
    d3[i] = h3[i] > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    float a = 0.f;
#pragma unroll
    for (int o = 0; o < 16; ++o) a = fmaf(P[OW3 + o * 32 + i], d3[o], a);
    d2[i] = h2[i] > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    float a = 0.f;
#pragma unroll
    for (int o = 0; o < 32; ++o) a = fmaf(P[OW2 + o * 64 + i], d2[o], a);
    d1[i] = h1[i] > 0.f ? a : 0.f;
  }
  float *g = part + (int64_t)blockIdx.x * NPARAM;
  const int t = threadIdx.x;
  // layer 5: d5 x h4
#pragma unroll
  for (int o = 0; o < 4; ++o) dl[t * 4 + o] = d5[o];
#pragma unroll
  for (int i = 0; i < 8; ++i) hl[t * 8 + i] = h4[i];
  __syncthreads();
  outer_reduce<4, 8>(dl, hl, nvalid, g + OW5, g + OB5);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 8; ++o) dl[t * 8 + o] = d4[o];
#pragma unroll
  for (int i = 0; i < 16; ++i) hl[t * 16 + i] = h3[i];
  __syncthreads();
  outer_reduce<8, 16>(dl, hl, nvalid, g + OW4, g + OB4);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 16; ++o) dl[t * 16 + o] = d3[o];
#pragma unroll
  for (int i = 0; i < 32; ++i) hl[t * 32 + i] = h2[i];
  __syncthreads();
  outer_reduce<16, 32>(dl, hl, nvalid, g + OW3, g + OB3);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 32; ++o) dl[t * 32 + o] = d2[o];
#pragma unroll
  for (int i = 0; i < 64; ++i) hl[t * 64 + i] = h1[i];
  __syncthreads();
  outer_reduce<32, 64>(dl, hl, nvalid, g + OW2, g + OB2);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 64; ++o) dl[t * 64 + o] = d1[o];
#pragma unroll
  for (int i = 0; i < 6; ++i) hl[t * 6 + i] = x0[i];
  __syncthreads();
  outer_reduce<64, 6>(dl, hl, nvalid, g + OW1, g + OB1);
  if (t == 0) {
    double a = 0.0;
    for (int k = 0; k < nvalid; ++k) a += (double)lsum[k];
    lpart[blockIdx.x] = a;
  }
}

// Deterministic two-level reduction of the partial rows (per-wave or
// per-block gradients and losses, in a fixed order) into the gradient, which
// is then written (mode 0) or takes one Adam step on the FP64 master
// parameters (mode 1).  Level 1: RSPLIT contiguous row ranges per parameter (and the loss as
// column NPARAM), in parallel; level 2 sums the RSPLIT values in order (64: 32
// and 128 were slower on batch 65536).
constexpr int RSPLIT = 64;

__global__ void __launch_bounds__(256)
k_reduce_rows(int nblk, const float *__restrict__ part, const double *__restrict__ lpart,
              double *__restrict__ part2) {
  const int i = blockIdx.x * 256 + threadIdx.x;  // parameter, NPARAM: the loss
  const int sp = blockIdx.y;
  if (i > NPARAM) return;
  const int b0 = (int)((int64_t)nblk * sp / RSPLIT), b1 = (int)((int64_t)nblk * (sp + 1) / RSPLIT);
  double g = 0.0;
  if (i < NPARAM) {
    for (int b = b0; b < b1; ++b) g += (double)part[(int64_t)b * NPARAM + i];
  } else {
    for (int b = b0; b < b1; ++b) g += lpart[b];
  }
  part2[(int64_t)sp * (NPARAM + 1) + i] = g;
}

__global__ void __launch_bounds__(256)
k_reduce_adam(const double *__restrict__ part2, double *__restrict__ P, double *__restrict__ am,
              double *__restrict__ av, double *__restrict__ grad, double *__restrict__ loss,
              double loss_scale, int mode, int accumulate_loss, double lr, double b1, double b2,
              double eps, double c1, double c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && loss) {
    double a = 0.0;
    for (int b = 0; b < RSPLIT; ++b) a += part2[(int64_t)b * (NPARAM + 1) + NPARAM];
    *loss = (accumulate_loss ? *loss : 0.0) + a * loss_scale;
  }
  if (i >= NPARAM) return;
  double g = 0.0;
  for (int b = 0; b < RSPLIT; ++b) g += part2[(int64_t)b * (NPARAM + 1) + i];
  if (mode == 0) {
    grad[i] = g;
    return;
  }
  const double m = b1 * am[i] + (1.0 - b1) * g;
  const double v = b2 * av[i] + (1.0 - b2) * g * g;
  am[i] = m;
  av[i] = v;
  P[i] = P[i] - lr * (m / c1) / (sqrt(v / c2) + eps);
}

__global__ void __launch_bounds__(256) k_to_f32(const double *__restrict__ P, float *__restrict__ P32) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < NPARAM) P32[i] = (float)P[i];
}

struct TrainWs {
  float *P32;
  void *tabs;
  float *part;
  double *lpart;
  double *part2;  // [RSPLIT][NPARAM + 1] level-1 sums
  size_t bytes;
};

int64_t partial_rows(int64_t batch) {
  const int64_t nblk = (batch + TB - 1) / TB;
  const int64_t nw = train_mfma_waves(batch);
  return nblk > nw ? nblk : nw;
}

TrainWs carve(void *ws, int32_t batch) {
  const int64_t rows = partial_rows(batch);
  char *b = (char *)ws;
  size_t off = 0;
  auto take = [&](size_t n) {
    char *p = b ? b + off : nullptr;
    off = (off + n + 255) & ~(size_t)255;
    return p;
  };
  TrainWs w;
  w.P32 = (float *)take(sizeof(float) * NPARAM);
  w.tabs = take(train_mfma_tab_bytes());
  w.part = (float *)take(sizeof(float) * NPARAM * (size_t)rows);
  w.lpart = (double *)take(sizeof(double) * (size_t)rows);
  w.part2 = (double *)take(sizeof(double) * (size_t)RSPLIT * (NPARAM + 1));
  w.bytes = off;
  return w;
}

}  // namespace

size_t train_workspace_bytes(int32_t batch) { return carve(nullptr, batch).bytes; }

bool train_precision_supported(int precision) { return precision == 1 || precision == 2; }

// Partial gradients of one mini-batch; returns the number of partial rows.
static hipError_t grad_pass(const double *P, const float *s, const uint8_t *y, const int64_t *idx,
                            int64_t mb, int precision, const TrainWs &w, int *rows, hipStream_t st) {
  if (precision == 2) {
    *rows = train_mfma_waves(mb);
    return launch_grad_mfma(P, w.tabs, s, y, idx, mb, w.part, w.lpart, st);
  }
  hipLaunchKernelGGL(k_to_f32, dim3((NPARAM + 255) / 256), dim3(256), 0, st, P, w.P32);
  const int64_t nblk = (mb + TB - 1) / TB;
  *rows = (int)nblk;
  hipLaunchKernelGGL(k_grad_f32, dim3((unsigned)nblk), dim3(TB), 0, st, w.P32, s, y, idx, mb,
                     (float)(1.0 / (double)mb), w.part, w.lpart);
  return hipGetLastError();
}

hipError_t launch_train_batch(double *P, double *m, double *v, int64_t step, const float *s,
                              const uint8_t *y, const int64_t *idx, int64_t mb, double lr,
                              double b1, double b2, double eps, int precision, double *loss_out,
                              double loss_scale, bool first, void *ws, hipStream_t st) {
  const TrainWs w = carve(ws, (int32_t)mb);
  int rows = 0;
  hipError_t e = grad_pass(P, s, y, idx, mb, precision, w, &rows, st);
  if (e != hipSuccess) return e;
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  hipLaunchKernelGGL(k_reduce_rows, dim3((NPARAM + 1 + 255) / 256, RSPLIT), dim3(256), 0, st, rows,
                     w.part, w.lpart, w.part2);
  hipLaunchKernelGGL(k_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, w.part2, P, m, v,
                     nullptr, loss_out, loss_scale, 1, first ? 0 : 1, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_grad(const double *P, const float *s, const uint8_t *y, int64_t n, int precision,
                       double *grad, double *loss, void *ws, hipStream_t st) {
  const TrainWs w = carve(ws, (int32_t)n);
  int rows = 0;
  hipError_t e = grad_pass(P, s, y, nullptr, n, precision, w, &rows, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_rows, dim3((NPARAM + 1 + 255) / 256, RSPLIT), dim3(256), 0, st, rows,
                     w.part, w.lpart, w.part2);
  hipLaunchKernelGGL(k_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, w.part2, nullptr,
                     nullptr, nullptr, grad, loss, 1.0 / (double)n, 0, 0, 0.0, 0.0, 0.0, 0.0, 1.0,
                     1.0);
  return hipGetLastError();
}

}  // namespace n6
