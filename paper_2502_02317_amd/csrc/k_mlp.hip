// Proposal network: forward pass, cross-entropy gradient and Adam (FP32).
//
// Gradient layout follows the parameters: W1 [H][F], b1 [H], w2 [H], b2,
// then the loss.  Each wavefront takes parents in a fixed grid-stride order
// with lane h owning hidden unit h, so every lane accumulates the gradient of
// its own parameters; waves and then blocks are summed in a fixed order, so
// the result does not depend on scheduling.
#include <cmath>

#include "mlp_dev.h"
#include "spg_internal.h"

namespace spg {

namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int kWaves = 4;
constexpr int kGradBlocks = 256;

// log p^(s | b) = log-softmax over s of the logits, one wavefront per parent.
__global__ __launch_bounds__(256) void k_mlp_fwd(int n, int d, const float *feats,
                                                 const float *prm, int H, float *logp) {
  __shared__ float P[kMaxHidden * (kFeat + 2) + 1];
  const int np = mlp_n_params(H);
  for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = prm[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * kWaves + w;
  if (b >= n) return;                       // no barrier below
  float lg[4];
  float mx = -INFINITY;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    lg[j] = -INFINITY;
    if (s < d) {
      lg[j] = mlp_logit(P, H, feats + ((long)b * d + s) * kFeat);
      mx = fmaxf(mx, lg[j]);
    }
  }
  mx = wave_max_f(mx);
  float se = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (lane + 64 * j < d) se += expf(lg[j] - mx);
  const float lse = mx + logf(wave_sum_f(se));
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    if (s < d) logp[(long)b * d + s] = lg[j] - lse;
  }
}

// Per-block partial gradients and loss, partial [gridDim.x][P + 1].
__global__ __launch_bounds__(256) void k_mlp_grad(int n, int d, const float *feats,
                                                  const float *target, const float *prm, int H,
                                                  float inv_n, float *partial) {
  __shared__ float P[kMaxHidden * (kFeat + 2) + 1];
  __shared__ float part[kWaves][kMaxHidden * (kFeat + 2) + 2];
  const int np = mlp_n_params(H);
  for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = prm[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool own = lane < H;
  const int h = own ? lane : 0;
  const float *W1 = P, *b1 = P + H * kFeat, *w2 = b1 + H;
  const float b2 = w2[H];
  float gW1[kFeat] = {0, 0, 0, 0, 0, 0};
  float gb1 = 0.0f, gw2 = 0.0f, gb2 = 0.0f, loss = 0.0f;
  const int stride = gridDim.x * kWaves;
  for (int b = blockIdx.x * kWaves + w; b < n; b += stride) {
    const float *fb = feats + (long)b * d * kFeat;
    const float *tb = target + (long)b * d;
    // logits; lane l keeps those of s = l + 64 j
    float lg[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int l = 0; l < 64; ++l) {
        const int s = 64 * j + l;
        if (s >= d) break;
        float a = b1[h];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) a = fmaf(W1[h * kFeat + k], fb[s * kFeat + k], a);
        const float v = own ? w2[h] * fmaxf(a, 0.0f) : 0.0f;
        const float lgt = wave_sum_f(v) + b2;
        if (lane == l) lg[j] = lgt;
      }
    float mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j) mx = fmaxf(mx, lg[j]);
    mx = wave_max_f(mx);
    float se = 0.0f, pt[4], pts = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = lane + 64 * j;
      pt[j] = 0.0f;
      if (s < d) {
        se += expf(lg[j] - mx);
        pt[j] = expf(tb[s]);
        pts += pt[j];
      }
    }
    const float lse = mx + logf(wave_sum_f(se));
    pts = wave_sum_f(pts);
    float dl[4], lsum = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = lane + 64 * j;
      dl[j] = 0.0f;
      if (s < d) {
        const float lp = lg[j] - lse;
        dl[j] = (expf(lp) * pts - pt[j]) * inv_n;
        if (pt[j] > 0.0f) lsum -= pt[j] * lp;
      }
    }
    loss += wave_sum_f(lsum) * inv_n;
    // backward: one child at a time, its dlogit broadcast from its lane
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int l = 0; l < 64; ++l) {
        const int s = 64 * j + l;
        if (s >= d) break;
        const float g = __shfl(dl[j], l);
        float a = b1[h];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) a = fmaf(W1[h * kFeat + k], fb[s * kFeat + k], a);
        gw2 = fmaf(g, fmaxf(a, 0.0f), gw2);
        const float dp = (a > 0.0f) ? g * w2[h] : 0.0f;
        gb1 += dp;
#pragma unroll
        for (int k = 0; k < kFeat; ++k) gW1[k] = fmaf(dp, fb[s * kFeat + k], gW1[k]);
        gb2 += g;
      }
  }
  if (own) {
    for (int k = 0; k < kFeat; ++k) part[w][h * kFeat + k] = gW1[k];
    part[w][H * kFeat + h] = gb1;
    part[w][H * kFeat + H + h] = gw2;
  }
  if (lane == 0) {
    part[w][H * kFeat + 2 * H] = gb2;
    part[w][np] = loss;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= np; i += blockDim.x) {
    float acc = 0.0f;
    for (int v = 0; v < kWaves; ++v) acc += part[v][i];
    partial[(long)blockIdx.x * (np + 1) + i] = acc;
  }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(int nb, int np, const float *partial,
                                                    float *grad, float *loss, float *loss_acc) {
  for (int i = threadIdx.x; i <= np; i += blockDim.x) {
    float acc = 0.0f;
    for (int k = 0; k < nb; ++k) acc += partial[(long)k * (np + 1) + i];
    if (i < np) {
      grad[i] = acc;
    } else {
      if (loss) *loss = acc;
      if (loss_acc) *loss_acc += acc;
    }
  }
}

// Adam (Kingma & Ba 2015); bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void k_adam(int np, float *prm, float *m, float *v, const float *g, float lr,
                       float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  prm[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

__global__ void k_to_float(long n, const double *src, float *dst) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

inline int grad_blocks(int n) {
  const int b = (int)nblk(n, kWaves);
  return b < kGradBlocks ? b : kGradBlocks;
}

}  // namespace

void mlp_forward(int n_beam, int d, const float *feats, const float *prm, int H, float *logp,
                 hipStream_t s) {
  bc_single("mlp_forward");
  if (n_beam <= 0) return;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk(n_beam, kWaves)), dim3(256), 0, s, n_beam, d, feats,
                     prm, H, logp);
  SPG_CHECK_LAUNCH();
}

size_t mlp_partial_floats(int H) { return (size_t)kGradBlocks * (mlp_n_params(H) + 1); }

void mlp_loss_grad(int n_beam, int d, const float *feats, const float *target, const float *prm,
                   int H, float *partial, float *grad, float *loss, float *loss_acc,
                   hipStream_t s) {
  bc_single("mlp_loss_grad");
  KTimer kt_("mlp_grad", s, 4.0 * n_beam * d * (kFeat * H + 2 * H));
  const int nb = grad_blocks(n_beam);
  if (nb > 0) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, n_beam, d, feats, target, prm, H,
                       1.0f / (float)n_beam, partial);
    SPG_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(256), 0, s, nb, mlp_n_params(H), partial, grad,
                     loss, loss_acc);
  SPG_CHECK_LAUNCH();
}

void mlp_adam(int P, float *prm, float *m, float *v, const float *grad, float lr, float bc1,
              float bc2, hipStream_t s) {
  bc_single("mlp_adam");
  hipLaunchKernelGGL(k_adam, dim3(nblk(P, 256)), dim3(256), 0, s, P, prm, m, v, grad, lr, bc1,
                     bc2);
  SPG_CHECK_LAUNCH();
}

void to_float(long n, const double *src, float *dst, hipStream_t s) {
  bc_single("to_float");
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_float, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
  SPG_CHECK_LAUNCH();
}

}  // namespace spg
