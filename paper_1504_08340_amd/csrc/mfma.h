// Interior stiffness K_RD u (first term of (3a)) as small dense contractions on
// the matrix cores (MFMA), FP32 state.
//
// For one brick and one displacement component u_i (27 nodal values), the 81
// values of d_k u_i at the 27 LGL points are B u_i with the fixed reference
// matrix B (81 x 27): row 27 k + q, column a holds D(q_k, a_k) when a and q
// agree on the two other axes, else 0 (D: derivative of the 1D quadratic
// basis at the LGL points).  A workgroup takes a tile of bricks and one
// source, and forms
//   G = B U,   U = [u_i of every brick and component]      (27 x 48)
//   S = w (lam tr(e) I + 2 mu e) at every point            (pointwise)
//   R = B^T S                                               (27 x 48)
// then sums R into the tile's nodes and stores them like the scalar kernel.
// The entries of B (0, +-1/2, +-3/2, +-2) are exact in BF16, so the BF16
// variant splits only the FP32 operand U (or S) into three BF16 parts
// (hi + mid + lo, 24 significant bits in all) and accumulates the three
// products in FP32.
#pragma once
#include "kernels.h"

namespace pmlfwi {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

enum { MFMA_F32 = 1, MFMA_BF16X3 = 3 };

// Threads of a matrix-core workgroup (its waves take the 16x16 output tiles in
// turn): 8 waves for FP32, 4 for the split BF16 form (145 VGPRs).
constexpr int mfma_threads(int mode) { return mode == MFMA_BF16X3 ? 256 : 512; }

// B[r][a]: derivative of local basis a along axis r / 27 at point r % 27.
__device__ __forceinline__ float bref(int r, int a) {
  if (r >= 81 || a >= 27) return 0.0f;
  const int d = r / 27, q = r - 27 * d;
  const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
  const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
  if (d == 0) return (ay == qy && az == qz) ? dlgl(qx, ax) : 0.0f;
  if (d == 1) return (ax == qx && az == qz) ? dlgl(qy, ay) : 0.0f;
  return (ax == qx && ay == qy) ? dlgl(qz, az) : 0.0f;
}

// Round-to-nearest-even FP32 -> BF16 (bit pattern), finite inputs.
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }

// Three BF16 parts whose sum carries the 24 bits of x.
__device__ __forceinline__ void split3(float x, short& hi, short& mid, short& lo) {
  const unsigned short h = bf16_bits(x);
  const float r1 = x - bf16_value(h);
  const unsigned short m = bf16_bits(r1);
  const float r2 = r1 - bf16_value(m);
  hi = (short)h;
  mid = (short)m;
  lo = (short)bf16_bits(r2);
}

// One 16x16 output tile of C = A (M x K) * Bm (K x N), A given by fa(row, k)
// and Bm by fb(k, col), accumulated in FP32 on the matrix cores.  Lane l of
// the wave supplies A[row0 + l % 16][k] and Bm[k][col0 + l % 16] for its k
// slots and receives C[row0 + 4 (l / 16) + r][col0 + l % 16], r = 0..3.
template <int MODE, int KMAX, typename FA, typename FB>
__device__ __forceinline__ v4f mfma_tile(int row0, int col0, FA fa, FB fb) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
  if constexpr (MODE == MFMA_F32) {
    for (int k0 = 0; k0 < KMAX; k0 += 4) {
      const int k = k0 + g;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa(row0 + i, k), fb(k, col0 + i), acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < KMAX; k0 += 16) {
      v4s a, bh, bm, bl;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * g + j;
        a[j] = (short)bf16_bits(fa(row0 + i, k));     // exact: entries of B
        short h, m, l;
        split3(fb(k, col0 + i), h, m, l);
        bh[j] = h;
        bm[j] = m;
        bl[j] = l;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bl, acc, 0, 0, 0);
    }
  }
  return acc;
}

// r_u += K_RD u for the x1 displacement of the input register, bricks of the
// tile list, one source per workgroup (blockIdx.y); mfma_threads(MODE) threads.
template <int MODE, int TX, int TY, int TZ>
__global__ void __launch_bounds__(mfma_threads(MODE))
interior_mfma_kernel(Geo g, const Tile* __restrict__ tiles, int ntiles, const float* __restrict__ Ybase,
                     long long ystride, const float* __restrict__ lam, const float* __restrict__ mu,
                     float* __restrict__ rbase, Part PT) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NE = TX * TY * TZ, NC = 3 * NE;   // columns: brick x component
  constexpr int MT_G = 6, NT = (NC + 15) / 16, MT_R = 2;              // 16x16 tiles of G (96 rows), R (32 rows)
  __shared__ float sU[3][NB];
  __shared__ float sLam[NB], sMu[NB];
  __shared__ float sG[81][NC];     // gradients, then the weighted stresses S in place
  __shared__ float sR[27][NC];

  const int ti = xcd_tile();
  if (ti >= ntiles) return;
  const Tile t = tiles[ti];
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const int nbx = 2 * cx + 1, nby = 2 * cy + 1, nbz = 2 * cz + 1;
  const size_t nn = (size_t)g.sn;
  const int src = blockIdx.y;
  const float* Yu = Ybase + (size_t)src * ystride;
  const float s2h = float(2.0 / g.h);

  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    const bool in = lx < nbx && ly < nby && lz < nbz;
    const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
    if (in) {
      const int mi = interior_index(g, i, j, k);
      const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
      sLam[n] = lam[mi];
      sMu[n] = mu[mi];
#pragma unroll
      for (int d = 0; d < 3; ++d) sU[d][n] = Yu[u_at(nn, d, node)];
    } else {
      sLam[n] = 0.0f;
      sMu[n] = 0.0f;
#pragma unroll
      for (int d = 0; d < 3; ++d) sU[d][n] = 0.0f;
    }
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  auto col_brick = [&](int c, int& ea, int& eb, int& ec) {
    const int e = c / 3;
    ea = e % TX;
    eb = (e / TX) % TY;
    ec = e / (TX * TY);
    return ea < cx && eb < cy && ec < cz;
  };
  // G = B U
  for (int tile = wave; tile < MT_G * NT; tile += mfma_threads(MODE) / 64) {
    const int mt = tile % MT_G, nt = tile / MT_G;
    auto fa = [&](int r, int a) { return bref(r, a); };
    auto fb = [&](int a, int c) -> float {
      int ea, eb, ec;
      if (a >= 27 || c >= NC || !col_brick(c, ea, eb, ec)) return 0.0f;
      const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
      return sU[c % 3][(2 * ea + ax) + BX * ((2 * eb + ay) + BY * (2 * ec + az))];
    };
    const v4f d = mfma_tile<MODE, MODE == MFMA_F32 ? 28 : 32>(16 * mt, 16 * nt, fa, fb);
    const int c = 16 * nt + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * mt + 4 * (lane >> 4) + r;
      if (row < 81 && c < NC) sG[row][c] = d[r];
    }
  }
  __syncthreads();

  // weighted stress at every point of every brick, in place
  for (int pq = threadIdx.x; pq < NE * 27; pq += blockDim.x) {
    const int e = pq / 27, q = pq - 27 * e;
    const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
    const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
    float H[3][3];   // H[i][k] = d_k u_i
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) H[i][k] = s2h * sG[27 * k + q][3 * e + i];
    const int nq = (2 * ea + qx) + BX * ((2 * eb + qy) + BY * (2 * ec + qz));
    const float la = sLam[nq], m = sMu[nq];
    const float wq = float(0.125 * g.h * g.h * g.h * wlgl(qx) * wlgl(qy) * wlgl(qz)) * s2h;
    const float tr = H[0][0] + H[1][1] + H[2][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float sik = (i == k ? la * tr : 0.0f) + m * (H[i][k] + H[k][i]);
        sG[27 * k + q][3 * e + i] = wq * sik;
      }
  }
  __syncthreads();

  // R = B^T S
  for (int tile = wave; tile < MT_R * NT; tile += mfma_threads(MODE) / 64) {
    const int mt = tile % MT_R, nt = tile / MT_R;
    auto fa = [&](int a, int r) { return bref(r, a); };
    auto fb = [&](int r, int c) -> float { return (r < 81 && c < NC) ? sG[r][c] : 0.0f; };
    const v4f d = mfma_tile<MODE, MODE == MFMA_F32 ? 84 : 96>(16 * mt, 16 * nt, fa, fb);
    const int c = 16 * nt + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * mt + 4 * (lane >> 4) + r;
      if (row < 27 && c < NC) sR[row][c] = d[r];
    }
  }
  __syncthreads();

  float* res = rbase + (size_t)src * PT.per_src;
  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    if (lx >= nbx || ly >= nby || lz >= nbz) continue;
    const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
    if (is_dirichlet(g, i, j, k)) continue;
    int exs[2], pxs[2], eys[2], pys[2], ezs[2], pzs[2];
    const int nex = node_bricks(lx, cx, exs, pxs);
    const int ney = node_bricks(ly, cy, eys, pys);
    const int nez = node_bricks(lz, cz, ezs, pzs);
    float r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
    for (int a3 = 0; a3 < 2; ++a3)
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int a1 = 0; a1 < 2; ++a1) {
          if (a1 >= nex || a2 >= ney || a3 >= nez) continue;
          const int e = exs[a1] + TX * (eys[a2] + TY * ezs[a3]);
          const int a = pxs[a1] + 3 * pys[a2] + 9 * pzs[a3];
          r0 += sR[a][3 * e + 0];
          r1 += sR[a][3 * e + 1];
          r2 += sR[a][3 * e + 2];
        }
    const int c = (lx == 2 * cx) | ((ly == 2 * cy) << 1) | ((lz == 2 * cz) << 2);
    const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
    const RowAddr ra = row_addr(g, PT, c, i, j, k, node, 0);
    res[ra.u] = r0;
    res[ra.u + 1] = r1;
    res[ra.u + 2] = r2;
  }
}

}  // namespace pmlfwi
