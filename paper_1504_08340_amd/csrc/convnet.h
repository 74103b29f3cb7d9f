// Kernels of the learned warm start: a small 3D convolutional network that
// maps surface traces to a coarse (lam, mu) perturbation, trained on traces
// the forward solver produces.  FP32, NCDHW layout (batch, channel, then the
// three spatial axes with the last fastest), cubic kernels of size 1 or 3
// with zero padding K/2, per-axis strides, optional ReLU after the bias.
// Every reduction runs in a fixed order (no atomics), so training is
// reproducible bit for bit.
#pragma once
#include <hip/hip_runtime.h>

#include "mfma.h"

namespace pmlfwi {

struct ConvShape {
  int N, Ci, D, H, W;      // input
  int Co, K;               // output channels, kernel size (1 or 3)
  int sd, sh, sw;          // strides
  int Do, Ho, Wo;          // output
};

__host__ __device__ inline int conv_out(int n, int K, int s) { return (n + 2 * (K / 2) - K) / s + 1; }

// y = act(b + w * x)
__global__ void __launch_bounds__(256) conv3d_forward_kernel(ConvShape c, const float* __restrict__ x,
                                                             const float* __restrict__ w,
                                                             const float* __restrict__ b, int relu,
                                                             float* __restrict__ y) {
  const long long total = (long long)c.N * c.Co * c.Do * c.Ho * c.Wo;
  const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= total) return;
  long long t = o;
  const int ow = (int)(t % c.Wo); t /= c.Wo;
  const int oh = (int)(t % c.Ho); t /= c.Ho;
  const int od = (int)(t % c.Do); t /= c.Do;
  const int co = (int)(t % c.Co);
  const int n = (int)(t / c.Co);
  const int p = c.K / 2, KK = c.K * c.K * c.K;
  float acc = b ? b[co] : 0.0f;
  for (int ci = 0; ci < c.Ci; ++ci) {
    const float* xc = x + ((long long)n * c.Ci + ci) * c.D * c.H * c.W;
    const float* wc = w + ((long long)co * c.Ci + ci) * KK;
    for (int kd = 0; kd < c.K; ++kd) {
      const int id = od * c.sd + kd - p;
      if (id < 0 || id >= c.D) continue;
      for (int kh = 0; kh < c.K; ++kh) {
        const int ih = oh * c.sh + kh - p;
        if (ih < 0 || ih >= c.H) continue;
        for (int kw = 0; kw < c.K; ++kw) {
          const int iw = ow * c.sw + kw - p;
          if (iw < 0 || iw >= c.W) continue;
          acc += wc[(kd * c.K + kh) * c.K + kw] * xc[((long long)id * c.H + ih) * c.W + iw];
        }
      }
    }
  }
  y[o] = (relu && acc < 0.0f) ? 0.0f : acc;
}

// ---- BF16 inference on the matrix cores -----------------------------------
// The convolution as an implicit GEMM: C[co][p] = sum_k W[co][k] X[k][p] with
// k = (ci, kd, kh, kw) and p the output position of one batch entry; W is
// the BF16 weight tensor read as a [Co][Ci K^3] matrix, X the zero-padded
// input patch gathered on the fly (im2col without a buffer).  One wave per 16
// output positions and every 16-row tile of output channels, v_mfma 16x16x16
// BF16 with FP32 accumulation; bias and ReLU in FP32, output rounded to BF16
// (hidden layers) or kept FP32 (the head).
__global__ void to_bf16_kernel(long long n, const float* __restrict__ in, unsigned short* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = bf16_bits(in[i]);
}

constexpr int CONV_MFMA_THREADS = 256;   // 4 waves, 64 output positions per workgroup

__global__ void __launch_bounds__(CONV_MFMA_THREADS)
conv3d_bf16_mfma_kernel(ConvShape c, const unsigned short* __restrict__ x, const unsigned short* __restrict__ w,
                        const float* __restrict__ b, int relu, int out_fp32, void* __restrict__ y) {
  const int P = c.Do * c.Ho * c.Wo;
  const int KK = c.K * c.K * c.K, Kdim = c.Ci * KK, pad = c.K / 2;
  const int n = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int col0 = blockIdx.x * 64 + wave * 16;
  const int p = col0 + i;                        // this lane's output position (B column)
  const bool pin = p < P;
  const int ow = pin ? p % c.Wo : 0, oh = pin ? (p / c.Wo) % c.Ho : 0, od = pin ? p / (c.Wo * c.Ho) : 0;
  const unsigned short* xn = x + (size_t)n * c.Ci * c.D * c.H * c.W;
  const int nrt = (c.Co + 15) / 16;
  for (int rt = 0; rt < nrt; ++rt) {
    const int row = rt * 16 + i;                 // this lane's A row (output channel)
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < Kdim; k0 += 16) {
      v4s a, bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * g + j;
        a[j] = (row < c.Co && k < Kdim) ? (short)w[(size_t)row * Kdim + k] : (short)0;
        short v = 0;
        if (pin && k < Kdim) {
          const int ci = k / KK, r = k - ci * KK;
          const int kd = r / (c.K * c.K), kh = (r / c.K) % c.K, kw = r % c.K;
          const int id = od * c.sd + kd - pad, ih = oh * c.sh + kh - pad, iw = ow * c.sw + kw - pad;
          if (id >= 0 && id < c.D && ih >= 0 && ih < c.H && iw >= 0 && iw < c.W)
            v = (short)xn[(((size_t)ci * c.D + id) * c.H + ih) * c.W + iw];
        }
        bb[j] = v;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
    }
    // lane holds C[rt*16 + 4 g + r][col0 + i], r = 0..3
    if (pin) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = rt * 16 + 4 * g + r;
        if (co >= c.Co) continue;
        float v = acc[r] + (b ? b[co] : 0.0f);
        if (relu && v < 0.0f) v = 0.0f;
        const size_t o = ((size_t)n * c.Co + co) * P + p;
        if (out_fp32) ((float*)y)[o] = v;
        else ((unsigned short*)y)[o] = bf16_bits(v);
      }
    }
  }
}

// g = dL/d(pre-activation) from dL/dy and, with ReLU, the activated output y.
__device__ __forceinline__ float pre_grad(const float* dy, const float* y, int relu, long long i) {
  return (relu && !(y[i] > 0.0f)) ? 0.0f : dy[i];
}

// dx = w^T * g  (gather form: every input element sums the outputs it feeds)
__global__ void __launch_bounds__(256) conv3d_backward_data_kernel(ConvShape c, const float* __restrict__ dy,
                                                                   const float* __restrict__ y, int relu,
                                                                   const float* __restrict__ w,
                                                                   float* __restrict__ dx) {
  const long long total = (long long)c.N * c.Ci * c.D * c.H * c.W;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  long long t = i;
  const int iw = (int)(t % c.W); t /= c.W;
  const int ih = (int)(t % c.H); t /= c.H;
  const int id = (int)(t % c.D); t /= c.D;
  const int ci = (int)(t % c.Ci);
  const int n = (int)(t / c.Ci);
  const int p = c.K / 2, KK = c.K * c.K * c.K;
  float acc = 0.0f;
  for (int co = 0; co < c.Co; ++co) {
    const long long ob = ((long long)n * c.Co + co) * c.Do * c.Ho * c.Wo;
    const float* wc = w + ((long long)co * c.Ci + ci) * KK;
    for (int kd = 0; kd < c.K; ++kd) {
      const int a = id + p - kd;
      if (a < 0 || a % c.sd) continue;
      const int od = a / c.sd;
      if (od >= c.Do) continue;
      for (int kh = 0; kh < c.K; ++kh) {
        const int bq = ih + p - kh;
        if (bq < 0 || bq % c.sh) continue;
        const int oh = bq / c.sh;
        if (oh >= c.Ho) continue;
        for (int kw = 0; kw < c.K; ++kw) {
          const int cq = iw + p - kw;
          if (cq < 0 || cq % c.sw) continue;
          const int ow = cq / c.sw;
          if (ow >= c.Wo) continue;
          const long long oi = ob + ((long long)od * c.Ho + oh) * c.Wo + ow;
          acc += wc[(kd * c.K + kh) * c.K + kw] * pre_grad(dy, y, relu, oi);
        }
      }
    }
  }
  dx[i] = acc;
}

// dw[co][ci][k] = sum over batch and outputs of g * x; one workgroup per
// weight, fixed-order tree reduction.
__global__ void __launch_bounds__(256) conv3d_backward_weight_kernel(ConvShape c, const float* __restrict__ dy,
                                                                     const float* __restrict__ y, int relu,
                                                                     const float* __restrict__ x,
                                                                     float* __restrict__ dw) {
  __shared__ float part[256];
  const int KK = c.K * c.K * c.K, p = c.K / 2;
  const int widx = blockIdx.x;
  const int k = widx % KK, ci = (widx / KK) % c.Ci, co = widx / (KK * c.Ci);
  const int kd = k / (c.K * c.K), kh = (k / c.K) % c.K, kw = k % c.K;
  const long long per = (long long)c.Do * c.Ho * c.Wo;
  float acc = 0.0f;
  for (long long t = threadIdx.x; t < (long long)c.N * per; t += blockDim.x) {
    const int n = (int)(t / per);
    long long r = t - n * per;
    const int ow = (int)(r % c.Wo); r /= c.Wo;
    const int oh = (int)(r % c.Ho);
    const int od = (int)(r / c.Ho);
    const int id = od * c.sd + kd - p, ih = oh * c.sh + kh - p, iw = ow * c.sw + kw - p;
    if (id < 0 || id >= c.D || ih < 0 || ih >= c.H || iw < 0 || iw >= c.W) continue;
    const long long oi = ((long long)n * c.Co + co) * per + ((long long)od * c.Ho + oh) * c.Wo + ow;
    acc += pre_grad(dy, y, relu, oi) * x[(((long long)n * c.Ci + ci) * c.D + id) * c.H * c.W + (long long)ih * c.W + iw];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) dw[widx] = part[0];
}

__global__ void __launch_bounds__(256) conv3d_backward_bias_kernel(ConvShape c, const float* __restrict__ dy,
                                                                   const float* __restrict__ y, int relu,
                                                                   float* __restrict__ db) {
  __shared__ float part[256];
  const int co = blockIdx.x;
  const long long per = (long long)c.Do * c.Ho * c.Wo;
  float acc = 0.0f;
  for (long long t = threadIdx.x; t < (long long)c.N * per; t += blockDim.x) {
    const int n = (int)(t / per);
    const long long oi = ((long long)n * c.Co + co) * per + (t - n * per);
    acc += pre_grad(dy, y, relu, oi);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = part[0];
}

// L = 1/(2n) sum (y - t)^2 over n entries; grad = (y - t)/n; one workgroup.
__global__ void __launch_bounds__(1024) mse_kernel(long long n, const float* __restrict__ y,
                                                   const float* __restrict__ t, float* __restrict__ loss,
                                                   float* __restrict__ grad) {
  __shared__ float part[1024];
  float acc = 0.0f;
  const float inv = 1.0f / (float)n;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const float r = y[i] - t[i];
    acc += r * r;
    if (grad) grad[i] = r * inv;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = 0.5f * part[0] * inv;
}

// Adam (Kingma and Ba, 2015) with bias correction; step t counts from 1.
__global__ void adam_kernel(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, int t) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mi = b1 * m[i] + (1.0f - b1) * g[i];
  const float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)t));
  const float vh = vi / (1.0f - powf(b2, (float)t));
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Network input from FP64 traces [nsrc][nsteps+1][nrec][3]: component comp at
// the receivers rec_idx[H*W] and steps t0 + t*tstride, t < T, times scale;
// out [nsrc][T][H][W] (one sample of the batch).
__global__ void trace_features_kernel(const double* __restrict__ traces, int nsrc, int nsteps, int nrec,
                                      const int* __restrict__ rec_idx, int HW, int T, int t0, int tstride,
                                      int comp, float scale, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nsrc * T * HW) return;
  const int r = (int)(i % HW);
  const int t = (int)((i / HW) % T);
  const int s = (int)(i / ((long long)HW * T));
  const long long step = (long long)t0 + (long long)t * tstride;
  out[i] = step <= nsteps
               ? scale * (float)traces[(((long long)s * (nsteps + 1) + step) * nrec + rec_idx[r]) * 3 + comp]
               : 0.0f;
}

// Coarse cell-centred field c[Dz][Gy][Gx] (cells of a regular grid over the
// closed interior box, z index 0 at the top) -> nodes of the closed interior:
// out = base * (1 + trilinear(c)), clamped to the cell centres at the edges.
__global__ void grid_to_nodes_kernel(const float* __restrict__ c, int Gx, int Gy, int Gz, int NIX, int NIY,
                                     int NIZ, const double* __restrict__ base, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NIX * NIY * NIZ) return;
  const int jz = j / (NIX * NIY), r = j - jz * NIX * NIY, jy = r / NIX, jx = r - jy * NIX;
  // node position in cell units: cell k spans [k, k+1), centre k + 1/2
  auto coord = [](int jn, int nn, int G, int& k0, float& f) {
    float u = (float)jn / (float)(nn - 1) * (float)G - 0.5f;
    u = fminf(fmaxf(u, 0.0f), (float)(G - 1));
    k0 = min((int)u, G - 2 >= 0 ? G - 2 : 0);
    f = G > 1 ? u - (float)k0 : 0.0f;
  };
  int cx0, cy0, cz0;
  float fx, fy, fz;
  coord(jx, NIX, Gx, cx0, fx);
  coord(jy, NIY, Gy, cy0, fy);
  coord(NIZ - 1 - jz, NIZ, Gz, cz0, fz);          // depth index from the top
  const int cx1 = min(cx0 + 1, Gx - 1), cy1 = min(cy0 + 1, Gy - 1), cz1 = min(cz0 + 1, Gz - 1);
  auto at = [&](int z, int y, int x) { return c[((long long)z * Gy + y) * Gx + x]; };
  const float v = (1 - fz) * ((1 - fy) * ((1 - fx) * at(cz0, cy0, cx0) + fx * at(cz0, cy0, cx1)) +
                              fy * ((1 - fx) * at(cz0, cy1, cx0) + fx * at(cz0, cy1, cx1))) +
                  fz * ((1 - fy) * ((1 - fx) * at(cz1, cy0, cx0) + fx * at(cz1, cy0, cx1)) +
                        fy * ((1 - fx) * at(cz1, cy1, cx0) + fx * at(cz1, cy1, cx1)));
  out[j] = base[j] * (1.0 + (double)v);
}

}  // namespace pmlfwi
