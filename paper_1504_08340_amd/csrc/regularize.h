// Control-problem terms on the closed interior (Sec. 3.1.3 and App. C), FP64.
//
//   Tikhonov (8):        R_TN(f) = 1/2 int |grad f|^2,        gradient (C.1b-c)
//   total variation (9): R_TV(f) = int (|grad f|^2 + eps)^1/2, gradient (C.1d-e)
//   M~ (C.1a):           lumped (LGL) mass of the closed interior, diagonal
//   (18):                g = M~^{-1} (g_mis + R g_reg)
//
// f is a nodal field on the closed-interior grid (id jx + NIX*(jy + NIY*jz)),
// integrals use the 3x3x3 LGL rule of every interior brick.  The TV
// denominator is evaluated pointwise at the LGL points, and the functional
// carries R rather than R/2 so that its derivative is the TV form of (17).
#pragma once
#include "geometry.h"

namespace pmlfwi {

__device__ __forceinline__ double dlgl64(int q, int a) {
  // derivative of 1D basis a at LGL point q (nodes -1, 0, 1)
  const double r0 = a == 0 ? -1.5 : (a == 1 ? 2.0 : -0.5);
  const double r1 = a == 0 ? -0.5 : (a == 1 ? 0.0 : 0.5);
  const double r2 = a == 0 ? 0.5 : (a == 1 ? -2.0 : 1.5);
  return q == 0 ? r0 : (q == 1 ? r1 : r2);
}
__device__ __forceinline__ double wlgl64(int a) { return a == 1 ? 4.0 / 3.0 : 1.0 / 3.0; }

enum { REG_TN = 0, REG_TV = 1 };

// grad f at LGL point q of the interior brick with lower node (x0, y0, z0).
__device__ __forceinline__ void point_grad(const Geo& g, const double* __restrict__ f, int x0, int y0, int z0,
                                           int qx, int qy, int qz, double G[3]) {
  const int sx = 1, sy = g.NIX, sz = g.NIX * g.NIY;
  const int base = (x0 + qx) * sx + (y0 + qy) * sy + (z0 + qz) * sz;
  double gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gx += dlgl64(qx, a) * f[base + (a - qx) * sx];
    gy += dlgl64(qy, a) * f[base + (a - qy) * sy];
    gz += dlgl64(qz, a) * f[base + (a - qz) * sz];
  }
  const double s = 2.0 / g.h;
  G[0] = s * gx;
  G[1] = s * gy;
  G[2] = s * gz;
}

// Quadrature term of the functional and the flux coefficient at one point.
__device__ __forceinline__ void point_terms(int kind, double eps, const double G[3], double w, double* val,
                                            double* coef) {
  const double s2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
  if (kind == REG_TN) {
    *val = 0.5 * w * s2;
    *coef = w;
  } else {
    const double r = sqrt(s2 + eps);
    *val = w * r;
    *coef = w / r;
  }
}

// Bricks of one axis that contain interior-closure index l: (brick, local position).
__device__ __forceinline__ int axis_bricks(int l, int ne, int* b, int* p) {
  if (l & 1) {
    b[0] = l >> 1;
    p[0] = 1;
    return 1;
  }
  int n = 0;
  if (l >= 2) {
    b[n] = (l >> 1) - 1;
    p[n] = 2;
    ++n;
  }
  if ((l >> 1) < ne) {
    b[n] = l >> 1;
    p[n] = 0;
    ++n;
  }
  return n;
}

// grad[j] = d R(f) / d f_j, gathered per node over the bricks that contain it
// (deterministic: no atomics).
__global__ void __launch_bounds__(256) reg_gradient_kernel(Geo g, int kind, double eps,
                                                           const double* __restrict__ f,
                                                           double* __restrict__ grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.n_int) return;
  const int jz = j / (g.NIX * g.NIY), r_ = j - jz * g.NIX * g.NIY, jy = r_ / g.NIX, jx = r_ - jy * g.NIX;
  int bx[2], px[2], by[2], py[2], bz[2], pz[2];
  const int nx = axis_bricks(jx, g.ex, bx, px), ny = axis_bricks(jy, g.ey, by, py),
            nz = axis_bricks(jz, g.ez, bz, pz);
  const double vol = 0.125 * g.h * g.h * g.h, s = 2.0 / g.h;
  double acc = 0.0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        const int x0 = 2 * bx[a], y0 = 2 * by[b], z0 = 2 * bz[c];
        const int p[3] = {px[a], py[b], pz[c]};
        // the points on the three lines through the node inside this brick
        for (int d = 0; d < 3; ++d)
          for (int q = 0; q < 3; ++q) {
            int qq[3] = {p[0], p[1], p[2]};
            qq[d] = q;
            double G[3], val, coef;
            point_grad(g, f, x0, y0, z0, qq[0], qq[1], qq[2], G);
            const double w = vol * wlgl64(qq[0]) * wlgl64(qq[1]) * wlgl64(qq[2]);
            point_terms(kind, eps, G, w, &val, &coef);
            acc += coef * G[d] * s * dlgl64(q, p[d]);
          }
      }
  grad[j] = acc;
}

// value[0] = R(f): one workgroup, fixed summation order (deterministic).
__global__ void __launch_bounds__(1024) reg_value_kernel(Geo g, int kind, double eps,
                                                         const double* __restrict__ f,
                                                         double* __restrict__ value) {
  __shared__ double part[1024];
  const long long npts = 27LL * g.ex * g.ey * g.ez;
  const double vol = 0.125 * g.h * g.h * g.h;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < npts; t += blockDim.x) {
    const int q = (int)(t % 27);
    const long long e = t / 27;
    const int ex = (int)(e % g.ex), ey = (int)((e / g.ex) % g.ey), ez = (int)(e / ((long long)g.ex * g.ey));
    const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
    double G[3], val, coef;
    point_grad(g, f, 2 * ex, 2 * ey, 2 * ez, qx, qy, qz, G);
    point_terms(kind, eps, G, vol * wlgl64(qx) * wlgl64(qy) * wlgl64(qz), &val, &coef);
    acc += val;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) value[0] = part[0];
}

// M~ diagonal (C.1a): interior lumped mass of every closed-interior node.
__global__ void material_mass_kernel(Geo g, double* __restrict__ m) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.n_int) return;
  const int jz = j / (g.NIX * g.NIY), r_ = j - jz * g.NIX * g.NIY, jy = r_ / g.NIX, jx = r_ - jy * g.NIX;
  double mrd, mp;
  lumped_masses_tab(g, jx + 2 * g.ps, jy + 2 * g.ps, jz + 2 * g.pb, mrd, mp);
  m[j] = mrd;
}

// (18): g = M~^{-1} (g_mis + R g_reg); g_reg may be null (R = 0).
__global__ void gradient_finalize_kernel(Geo g, const double* __restrict__ gmis, const double* __restrict__ greg,
                                         double R, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.n_int) return;
  const int jz = j / (g.NIX * g.NIY), r_ = j - jz * g.NIX * g.NIY, jy = r_ / g.NIX, jx = r_ - jy * g.NIX;
  double mrd, mp;
  lumped_masses_tab(g, jx + 2 * g.ps, jy + 2 * g.ps, jz + 2 * g.pb, mrd, mp);
  const double v = gmis[j] + (greg ? R * greg[j] : 0.0);
  out[j] = v / mrd;
}

// out[0] = sum_i a_i b_i (w_i): one workgroup, fixed order.
__global__ void __launch_bounds__(1024) dot_kernel(long long n, const double* __restrict__ a,
                                                   const double* __restrict__ b, const double* __restrict__ w,
                                                   double* __restrict__ out) {
  __shared__ double part[1024];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) acc += a[i] * b[i] * (w ? w[i] : 1.0);
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

// out = alpha x + beta y (y may be null when beta = 0; out may alias x or y):
// the vector updates of the optimizer (L-BFGS two-loop recursion, the model
// update (19), the biased direction (25), y = g1 - g).  FP64, elementwise.
__global__ void axpby_kernel(long long n, double alpha, const double* x, double beta, const double* y,
                             double* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = beta == 0.0 ? alpha * x[i] : alpha * x[i] + beta * y[i];
}

// out[0] = max_i |x_i| (one workgroup; max is exact, so any order gives the same bits).
__global__ void __launch_bounds__(1024) absmax_kernel(long long n, const double* __restrict__ x,
                                                      double* __restrict__ out) {
  __shared__ double part[1024];
  double m = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(x[i]));
  part[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

}  // namespace pmlfwi
