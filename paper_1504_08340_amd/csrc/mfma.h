// Interior stiffness K_RD u (first term of (3a)) and the PML operator (the
// remaining blocks of (3a)-(3b) on the PML bricks) as small dense contractions
// on the matrix cores (MFMA), FP32 state.
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
// The PML kernel uses the same B: its S-rows need the gradients of the three
// axis fields W_k (d_k W_k,i at the points: B_k W_k, B_k the 27 rows of axis
// k), its u-rows the contraction B^T of the weighted nodal tensor T.
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

// B in LDS, rows padded to 96 and columns to 32 with zeros, formed once per
// workgroup so the matrix-core loops read their A operand instead of forming
// it per lane and k step.
constexpr int BT_ROWS = 96, BT_COLS = 32;
__device__ __forceinline__ void fill_btab(float (&sB)[BT_ROWS][BT_COLS]) {
  for (int idx = threadIdx.x; idx < BT_ROWS * BT_COLS; idx += blockDim.x) {
    const int r = idx / BT_COLS, a = idx - BT_COLS * r;
    sB[r][a] = bref(r, a);
  }
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
  __shared__ float sB[BT_ROWS][BT_COLS];

  const int ti = xcd_tile();
  if (ti >= ntiles) return;
  const Tile t = tiles[ti];
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const int nbx = 2 * cx + 1, nby = 2 * cy + 1, nbz = 2 * cz + 1;
  fill_btab(sB);
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
    auto fa = [&](int r, int a) { return sB[r][a]; };
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
    auto fa = [&](int a, int r) { return sB[r][a]; };
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


// PML rows (forward, or transposed with ADJ) of the PML bricks of the tile list
// on the matrix cores, one row type per launch (PART: PML_SROWS or
// PML_UROWS), one source per workgroup (blockIdx.y), mfma_threads(MODE)
// threads.  The nodal fields W and T are those of the scalar PML kernel; then
//   S-rows:  G_k = B_k W_k (27 x 3 NE per axis k), Q at every point from
//            H_ik = (2/h) G_k[q][i] (with the materials when forward), and
//            every box node sums Q over its bricks;
//   u-rows:  R = B^T Tw, Tw[27 k + q][3 e + i] = w_q (2/h) T_ik at the box node
//            of point q of brick e, and every box node sums R over its bricks.
template <int MODE, int TX, int TY, int TZ, bool ADJ, int PART>
__global__ void __launch_bounds__(mfma_threads(MODE))
pml_mfma_kernel(Geo g, const Tile* __restrict__ tiles, int ntiles, const float* __restrict__ Ybase,
                long long ystride, const float* __restrict__ lam, const float* __restrict__ mu,
                float* __restrict__ rbase, Part PT) {
  constexpr bool DS = PART == PML_SROWS, DU = PART == PML_UROWS;
  static_assert(DS || DU, "one row type per launch");
  constexpr bool MATQ = DS && !ADJ;
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NE = TX * TY * TZ, NC = 3 * NE, NP = 27 * NE;
  constexpr int NT = (NC + 15) / 16;
  constexpr int NW = mfma_threads(MODE) / 64;
  constexpr int PER = (NP + mfma_threads(MODE) - 1) / mfma_threads(MODE);   // points per thread
  __shared__ float sF[9][NB];        // DS: W [3k + i];  DU: T [3i + k]
  __shared__ float sLam[MATQ ? NB : 1], sMu[MATQ ? NB : 1];
  __shared__ float sG[81][NC];       // DS: G, then Q as [6][NP];  DU: Tw
  __shared__ float sR[DU ? 27 : 1][DU ? NC : 1];
  __shared__ float sB[BT_ROWS][BT_COLS];
  static_assert(6 * NP <= 81 * NC, "Q fits in the gradient buffer");

  const int ti = xcd_tile();
  if (ti >= ntiles) return;
  const Tile t = tiles[ti];
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const size_t nn = (size_t)g.sn, np = (size_t)g.sp;
  const int src = blockIdx.y;
  const float* Y = Ybase + (size_t)src * ystride;
  const float s2h = float(2.0 / g.h);
  const double wh3 = 0.125 * g.h * g.h * g.h;
  fill_btab(sB);

  // phase 1: nodal fields of the box nodes (zero outside the tile)
  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    const bool live = lx <= 2 * cx && ly <= 2 * cy && lz <= 2 * cz;
    if (!live) {
#pragma unroll
      for (int c = 0; c < 9; ++c) sF[c][n] = 0.0f;
      if constexpr (MATQ) {
        sLam[n] = 0.0f;
        sMu[n] = 0.0f;
      }
      continue;
    }
    const int gi = 2 * t.x + lx, gj = 2 * t.y + ly, gk = 2 * t.z + lz;
    float Le[3], Lp[3], Lw[3], la = 0.0f, m = 0.0f;
    bool hist;
    size_t gnode, gp;
    pml_node_setup<float>(g, gi, gj, gk, Le, Lp, Lw, hist, gnode, gp);
    if constexpr (MATQ || (DU && ADJ)) {
      const int mi = material_index(g, gi, gj, gk);
      la = lam[mi];
      m = mu[mi];
      if constexpr (MATQ) {
        sLam[n] = la;
        sMu[n] = m;
      }
    }
    PmlNode<float> v;
    pml_load_node<float, DS, DU>(Y, nn, np, gnode, gp, hist, v);
    if constexpr (DS) pml_node_w<float, NB>(v, Le, Lp, Lw, n, sF);
    if constexpr (DU) pml_node_t<float, ADJ, NB>(v, Le, Lp, Lw, la, m, n, sF);
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
  auto box = [&](int ea, int eb, int ec, int q) {   // box node of point (or local node) q of a brick
    return (2 * ea + q % 3) + BX * ((2 * eb + (q / 3) % 3) + BY * (2 * ec + q / 9));
  };
  float* res = rbase + (size_t)src * PT.per_src;

  if constexpr (DS) {
    // G_k = B_k W_k: row tiles 2k, 2k + 1 hold the 27 rows of axis k
    for (int tile = wave; tile < 6 * NT; tile += NW) {
      const int mt = tile % 6, nt = tile / 6, k = mt >> 1;
      auto fa = [&](int r, int a) { return r < 27 ? sB[27 * k + r][a] : 0.0f; };
      auto fb = [&](int a, int c) -> float {
        int ea, eb, ec;
        if (a >= 27 || c >= NC || !col_brick(c, ea, eb, ec)) return 0.0f;
        return sF[3 * k + c % 3][box(ea, eb, ec, a)];
      };
      const v4f d = mfma_tile<MODE, MODE == MFMA_F32 ? 28 : 32>(16 * (mt & 1), 16 * nt, fa, fb);
      const int c = 16 * nt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (mt & 1) + 4 * (lane >> 4) + r;
        if (row < 27 && c < NC) sG[27 * k + row][c] = d[r];
      }
    }
    __syncthreads();
    // Q at every point of every brick (registers), then in place as [6][NP]
    float Qv[PER][6];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int pq = threadIdx.x + j * mfma_threads(MODE);
#pragma unroll
      for (int v = 0; v < 6; ++v) Qv[j][v] = 0.0f;
      if (pq >= NP) continue;
      const int e = pq / 27, q = pq - 27 * e;
      const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
      if (ea >= cx || eb >= cy || ec >= cz) continue;
      float H[3][3];   // H[i][k] = d_k W_k,i
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) H[i][k] = s2h * sG[27 * k + q][3 * e + i];
      const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
      const float wq = float(wh3 * wlgl(qx) * wlgl(qy) * wlgl(qz));
      if constexpr (!ADJ) {
        const int nq = box(ea, eb, ec, q);
        const float la = sLam[nq], m = sMu[nq];
        const float tr = H[0][0] + H[1][1] + H[2][2];
        Qv[j][0] = -wq * (la * tr + 2 * m * H[0][0]);
        Qv[j][1] = -wq * (la * tr + 2 * m * H[1][1]);
        Qv[j][2] = -wq * (la * tr + 2 * m * H[2][2]);
        Qv[j][3] = -wq * (m * (H[1][2] + H[2][1]));
        Qv[j][4] = -wq * (m * (H[0][2] + H[2][0]));
        Qv[j][5] = -wq * (m * (H[0][1] + H[1][0]));
      } else {
        Qv[j][0] = wq * H[0][0];
        Qv[j][1] = wq * H[1][1];
        Qv[j][2] = wq * H[2][2];
        Qv[j][3] = wq * (H[1][2] + H[2][1]);
        Qv[j][4] = wq * (H[0][2] + H[2][0]);
        Qv[j][5] = wq * (H[0][1] + H[1][0]);
      }
    }
    __syncthreads();
    float* sQ = &sG[0][0];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int pq = threadIdx.x + j * mfma_threads(MODE);
      if (pq < NP) {
#pragma unroll
        for (int v = 0; v < 6; ++v) sQ[v * NP + pq] = Qv[j][v];
      }
    }
    __syncthreads();
    for (int n = threadIdx.x; n < NB; n += blockDim.x) {
      const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
      if (lx > 2 * cx || ly > 2 * cy || lz > 2 * cz) continue;
      const int gi = 2 * t.x + lx, gj = 2 * t.y + ly, gk = 2 * t.z + lz;
      float q6[6];
      pml_s_rows<float, TX, TY, TZ>(cx, cy, cz, lx, ly, lz, sQ, q6);
      const size_t gnode = (size_t)gi + (size_t)g.NX * (gj + (size_t)g.NY * gk);
      const size_t gp = (size_t)pml_index(g, gi, gj, gk);
      const int cs = (lx == 2 * cx) | ((ly == 2 * cy) << 1) | ((lz == 2 * cz) << 2);
      const RowAddr ra = row_addr(g, PT, cs, gi, gj, gk, gnode, gp);
#pragma unroll
      for (int v = 0; v < 6; ++v) res[ra.s + v] = q6[v];
    }
  } else {
    // weighted nodal tensor at the points: Tw[27 k + q][3 e + i], one thread
    // per point of a brick (zero for bricks outside a ragged tile)
    for (int pq = threadIdx.x; pq < NP; pq += blockDim.x) {
      const int e = pq / 27, q = pq - 27 * e;
      const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
      const bool in = ea < cx && eb < cy && ec < cz;
      const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
      const float wq = in ? float(wh3 * wlgl(qx) * wlgl(qy) * wlgl(qz)) * s2h : 0.0f;
      const int nq = in ? box(ea, eb, ec, q) : 0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) sG[27 * k + q][3 * e + i] = wq * sF[3 * i + k][nq];
    }
    __syncthreads();
    // R = B^T Tw
    for (int tile = wave; tile < 2 * NT; tile += NW) {
      const int mt = tile % 2, nt = tile / 2;
      auto fa = [&](int a, int r) { return sB[r][a]; };
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
    for (int n = threadIdx.x; n < NB; n += blockDim.x) {
      const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
      if (lx > 2 * cx || ly > 2 * cy || lz > 2 * cz) continue;
      const int gi = 2 * t.x + lx, gj = 2 * t.y + ly, gk = 2 * t.z + lz;
      if (is_dirichlet(g, gi, gj, gk)) continue;
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
      const size_t gnode = (size_t)gi + (size_t)g.NX * (gj + (size_t)g.NY * gk);
      const size_t gp = (size_t)pml_index(g, gi, gj, gk);
      const int cs = (lx == 2 * cx) | ((ly == 2 * cy) << 1) | ((lz == 2 * cz) << 2);
      const RowAddr ra = row_addr(g, PT, cs, gi, gj, gk, gnode, gp);
      res[ra.u] = r0;
      res[ra.u + 1] = r1;
      res[ra.u + 2] = r2;
    }
  }
}

}  // namespace pmlfwi
