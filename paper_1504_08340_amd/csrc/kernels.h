// HIP kernels of the hot path (CDNA4 / gfx950).
//
//   interior_element_kernel : interior stiffness K_RD applied to a displacement
//                             field (first term of (3a)); optionally the
//                             Lame-parameter gradient terms (C.1f)-(C.1g).
//   pml_element_kernel      : PML coupling terms of (3a) (u-rows) and (3b)
//                             (S-rows), forward or transposed.
//   nodal_rk_kernel         : nodal PML terms, M^{-1}, classical RK4 stage
//                             combination of (6), source injection.
//
// Register layout (per source, type R): U part 6 x n_nodes
//   [x1 u_x, u_y, u_z | x2 u_x, u_y, u_z] on the full grid, then P part
//   21 x n_pml [x0 u (3) | x0 S (6) | x1 S (6) | x2 S (6)] on the PML shell.
//   Stress order (xx, yy, zz, yz, xz, xy).
// Residual layout (per source): 3 x n_nodes u-rows, then 6 x n_pml S-rows.
#pragma once
#include "geometry.h"

namespace pmlfwi {

enum { P_X0U = 0, P_X0S = 3, P_X1S = 9, P_X2S = 15, P_NCOMP = 21, U_NCOMP = 6 };

// Voigt slot of the symmetric pair (i, k).
__host__ __device__ constexpr int vidx(int i, int k) { return i == k ? i : 6 - i - k; }

// Derivative of 1D basis a at LGL point q: D[q][a] (nodes -1, 0, 1).
__device__ __forceinline__ double dlgl(int q, int a) {
  // rows q = 0: (-3/2, 2, -1/2); q = 1: (-1/2, 0, 1/2); q = 2: (1/2, -2, 3/2)
  const double r0 = a == 0 ? -1.5 : (a == 1 ? 2.0 : -0.5);
  const double r1 = a == 0 ? -0.5 : (a == 1 ? 0.0 : 0.5);
  const double r2 = a == 0 ? 0.5 : (a == 1 ? -2.0 : 1.5);
  return q == 0 ? r0 : (q == 1 ? r1 : r2);
}
__device__ __forceinline__ double wlgl(int a) { return a == 1 ? 4.0 / 3.0 : 1.0 / 3.0; }

struct Tile {  // bricks [x, x+cx) x [y, y+cy) x [z, z+cz)
  int x, y, z, c;  // c = cx | cy << 8 | cz << 16
};

// Per-dimension list of the bricks of a tile that contain local node l:
// (brick offset, position of the node in that brick).  At most two.
__device__ __forceinline__ int node_bricks(int l, int cnt, int* e, int* p) {
  if (l & 1) {
    e[0] = (l - 1) >> 1;
    p[0] = 1;
    return 1;
  }
  int n = 0;
  if (l >= 2) {
    e[n] = (l >> 1) - 1;
    p[n] = 2;
    ++n;
  }
  if ((l >> 1) < cnt) {
    e[n] = l >> 1;
    p[n] = 0;
    ++n;
  }
  return n;
}

template <typename R>
__device__ __forceinline__ void atomic_add(R* p, R v) {
  unsafeAtomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// Interior bricks: r_u += K_RD u  (u = x1 displacement of the input register).
// GRAD: also  g -= b_s * sum_e w|J| (div z div u_f, 2 eps(z):eps(u_f)) at the
// LGL nodes, z = the displacement read here, u_f = stored forward stage field.
template <typename R, int TX, int TY, int TZ, bool GRAD>
__global__ void __launch_bounds__(128)
interior_element_kernel(Geo g, const Tile* __restrict__ tiles, const R* __restrict__ Ybase,
                        long long ystride, const R* __restrict__ lam, const R* __restrict__ mu,
                        R* __restrict__ rbase, long long rstride, const R* __restrict__ fwd,
                        long long fstride, double gw, double* __restrict__ g_lam,
                        double* __restrict__ g_mu) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NP = 27 * TX * TY * TZ;
  __shared__ R sU[3][NB];
  __shared__ R sLam[NB], sMu[NB];
  __shared__ R sS[6][NP];
  __shared__ R sV[GRAD ? 3 : 1][GRAD ? NB : 1];
  __shared__ double sG[GRAD ? 2 : 1][GRAD ? NP : 1];

  const Tile t = tiles[blockIdx.x];
  const int src = blockIdx.y;
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const int nbx = 2 * cx + 1, nby = 2 * cy + 1, nbz = 2 * cz + 1;
  const size_t nn = (size_t)g.n_nodes;
  const R* Yu = Ybase + (size_t)src * ystride;
  R* res = rbase + (size_t)src * rstride;
  const R* F = GRAD ? fwd + (size_t)src * fstride : nullptr;

  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    if (lx >= nbx || ly >= nby || lz >= nbz) continue;
    const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
    const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
    const int mi = interior_index(g, i, j, k);
#pragma unroll
    for (int d = 0; d < 3; ++d) sU[d][n] = Yu[d * nn + node];
    sLam[n] = lam[mi];
    sMu[n] = mu[mi];
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < 3; ++d) sV[d][n] = F[(size_t)d * g.n_int + mi];
    }
  }
  __syncthreads();

  const R s2h = R(2.0 / g.h);
  for (int q = threadIdx.x; q < NP; q += blockDim.x) {
    const int pt = q % 27, e = q / 27;
    const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
    if (ea >= cx || eb >= cy || ec >= cz) continue;
    const int qa = pt % 3, qb = (pt / 3) % 3, qc = pt / 9;
    const int lx = 2 * ea + qa, ly = 2 * eb + qb, lz = 2 * ec + qc;
    const int nq = lx + BX * (ly + BY * lz);
    R G[3][3], Gf[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      R gx = 0, gy = 0, gz = 0, fx = 0, fy = 0, fz = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R cxa = R(dlgl(qa, a)), cya = R(dlgl(qb, a)), cza = R(dlgl(qc, a));
        const int nx = (2 * ea + a) + BX * (ly + BY * lz);
        const int ny = lx + BX * ((2 * eb + a) + BY * lz);
        const int nz = lx + BX * (ly + BY * (2 * ec + a));
        gx += cxa * sU[d][nx];
        gy += cya * sU[d][ny];
        gz += cza * sU[d][nz];
        if constexpr (GRAD) {
          fx += cxa * sV[d][nx];
          fy += cya * sV[d][ny];
          fz += cza * sV[d][nz];
        }
      }
      G[d][0] = gx * s2h; G[d][1] = gy * s2h; G[d][2] = gz * s2h;
      if constexpr (GRAD) { Gf[d][0] = fx * s2h; Gf[d][1] = fy * s2h; Gf[d][2] = fz * s2h; }
    }
    const R wq = R(0.125 * g.h * g.h * g.h * wlgl(qa) * wlgl(qb) * wlgl(qc));
    const R la = sLam[nq], m = sMu[nq];
    const R tr = G[0][0] + G[1][1] + G[2][2];
    sS[0][q] = wq * (la * tr + 2 * m * G[0][0]);
    sS[1][q] = wq * (la * tr + 2 * m * G[1][1]);
    sS[2][q] = wq * (la * tr + 2 * m * G[2][2]);
    sS[3][q] = wq * (m * (G[1][2] + G[2][1]));
    sS[4][q] = wq * (m * (G[0][2] + G[2][0]));
    sS[5][q] = wq * (m * (G[0][1] + G[1][0]));
    if constexpr (GRAD) {
      const double dz = (double)tr, du = (double)(Gf[0][0] + Gf[1][1] + Gf[2][2]);
      double ee = 2.0 * ((double)G[0][0] * Gf[0][0] + (double)G[1][1] * Gf[1][1] +
                         (double)G[2][2] * Gf[2][2]);
      ee += (double)(G[1][2] + G[2][1]) * (double)(Gf[1][2] + Gf[2][1]);
      ee += (double)(G[0][2] + G[2][0]) * (double)(Gf[0][2] + Gf[2][0]);
      ee += (double)(G[0][1] + G[1][0]) * (double)(Gf[0][1] + Gf[1][0]);
      sG[0][q] = (double)wq * dz * du;
      sG[1][q] = (double)wq * ee;
    }
  }
  __syncthreads();

  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    if (lx >= nbx || ly >= nby || lz >= nbz) continue;
    const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
    int exs[2], pxs[2], eys[2], pys[2], ezs[2], pzs[2];
    const int nex = node_bricks(lx, cx, exs, pxs);
    const int ney = node_bricks(ly, cy, eys, pys);
    const int nez = node_bricks(lz, cz, ezs, pzs);
    R r0 = 0, r1 = 0, r2 = 0;
    double gl = 0.0, gm = 0.0;
    for (int a3 = 0; a3 < nez; ++a3)
      for (int a2 = 0; a2 < ney; ++a2)
        for (int a1 = 0; a1 < nex; ++a1) {
          const int ea = exs[a1], eb = eys[a2], ec = ezs[a3];
          const int pa = pxs[a1], pb = pys[a2], pc = pzs[a3];
          const int eb0 = 27 * (ea + TX * (eb + TY * ec));
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const R cxa = R(dlgl(a, pa)), cya = R(dlgl(a, pb)), cza = R(dlgl(a, pc));
            const int qx = eb0 + a + 3 * pb + 9 * pc;
            const int qy = eb0 + pa + 3 * a + 9 * pc;
            const int qz = eb0 + pa + 3 * pb + 9 * a;
            r0 += cxa * sS[0][qx] + cya * sS[5][qy] + cza * sS[4][qz];
            r1 += cxa * sS[5][qx] + cya * sS[1][qy] + cza * sS[3][qz];
            r2 += cxa * sS[4][qx] + cya * sS[3][qy] + cza * sS[2][qz];
          }
          if constexpr (GRAD) {
            const int qn = eb0 + pa + 3 * pb + 9 * pc;
            gl += sG[0][qn];
            gm += sG[1][qn];
          }
        }
    if (!is_dirichlet(g, i, j, k)) {
      const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
      atomic_add(&res[node], r0 * s2h);
      atomic_add(&res[nn + node], r1 * s2h);
      atomic_add(&res[2 * nn + node], r2 * s2h);
    }
    if constexpr (GRAD) {
      const int mi = interior_index(g, i, j, k);
      atomic_add(&g_lam[mi], gw * gl);
      atomic_add(&g_mu[mi], gw * gm);
    }
  }
}

// ---------------------------------------------------------------------------
// PML bricks.  Forward (ADJ = false), for the input register (x0, x1, x2):
//   u-rows:  r_u += int grad w~ : (S' Le + S Lp + Sbar Lw)
//   S-rows:  r_S -= int T~ : (mu (H + H^T) + lam tr(H) I),
//            H_ik = d/dx_k (Le_kk u'_i + Lp_kk u_i + Lw_kk ubar_i)
// Transposed (ADJ = true): the same blocks transposed, applied to the adjoint
// register (y0, y1, y2) in the slots of (x0, x1, x2):
//   u-rows:  r_u += int grad w~ : T',  T'_ik = -(mu (1+d_ik) Z_k,ik + lam d_ik tr Z_i),
//            Z_k = Le_kk T2 + Lp_kk T1 + Lw_kk T0 (symmetric stress-like fields)
//   S-rows:  r_S += int T~_ab (H_ab + H_ba)  (a != b),  H_aa  (a = b).
template <typename R, int TX, int TY, int TZ, bool ADJ>
__global__ void __launch_bounds__(128)
pml_element_kernel(Geo g, const Tile* __restrict__ tiles, const R* __restrict__ Ybase,
                   long long ystride, const R* __restrict__ lam, const R* __restrict__ mu,
                   R* __restrict__ rbase, long long rstride) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NP = 27 * TX * TY * TZ;
  __shared__ R sW[9][NB];   // [3k + i]: Le_kk u'_i + Lp_kk u_i + Lw_kk ubar_i
  __shared__ R sT[9][NB];   // [3i + k]: nodal stress-like tensor of the u-rows
  __shared__ R sLam[ADJ ? 1 : NB], sMu[ADJ ? 1 : NB];
  __shared__ R sQ[6][NP];

  const Tile t = tiles[blockIdx.x];
  const int src = blockIdx.y;
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const int nbx = 2 * cx + 1, nby = 2 * cy + 1, nbz = 2 * cz + 1;
  const size_t nn = (size_t)g.n_nodes, np = (size_t)g.n_pml;
  const R* Y = Ybase + (size_t)src * ystride;
  const R* P = Y + 6 * nn;
  R* res = rbase + (size_t)src * rstride;

  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    if (lx >= nbx || ly >= nby || lz >= nbz) continue;
    const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
    const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
    const size_t p = (size_t)pml_index(g, i, j, k);
    const PmlCoef c = pml_coef(g, i, j, k);
    const bool hist = c.nbeta >= 2;
    R u1[3], u2[3], u0[3], s0[6], s1[6], s2[6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u1[d] = Y[d * nn + node];
      u2[d] = Y[(3 + d) * nn + node];
      u0[d] = hist ? P[(P_X0U + d) * np + p] : R(0);
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      s1[v] = P[(P_X1S + v) * np + p];
      s2[v] = P[(P_X2S + v) * np + p];
      s0[v] = hist ? P[(P_X0S + v) * np + p] : R(0);
    }
    R Le[3], Lp[3], Lw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) { Le[d] = R(c.Le[d]); Lp[d] = R(c.Lp[d]); Lw[d] = R(c.Lw[d]); }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) sW[3 * kk + ii][n] = Le[kk] * u2[ii] + Lp[kk] * u1[ii] + Lw[kk] * u0[ii];
    const int mi = material_index(g, i, j, k);
    const R la = lam[mi], m = mu[mi];
    if constexpr (!ADJ) {
      sLam[n] = la;
      sMu[n] = m;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const int v = vidx(ii, kk);
          sT[3 * ii + kk][n] = Le[kk] * s2[v] + Lp[kk] * s1[v] + Lw[kk] * s0[v];
        }
    } else {
      const R t2 = s2[0] + s2[1] + s2[2], t1 = s1[0] + s1[1] + s1[2], t0 = s0[0] + s0[1] + s0[2];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const int v = vidx(ii, kk);
          const R z = Le[kk] * s2[v] + Lp[kk] * s1[v] + Lw[kk] * s0[v];
          R val = (ii == kk ? R(2) : R(1)) * m * z;
          if (ii == kk) val += la * (Le[ii] * t2 + Lp[ii] * t1 + Lw[ii] * t0);
          sT[3 * ii + kk][n] = -val;
        }
    }
  }
  __syncthreads();

  const R s2h = R(2.0 / g.h);
  for (int q = threadIdx.x; q < NP; q += blockDim.x) {
    const int pt = q % 27, e = q / 27;
    const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
    if (ea >= cx || eb >= cy || ec >= cz) continue;
    const int qa = pt % 3, qb = (pt / 3) % 3, qc = pt / 9;
    const int lx = 2 * ea + qa, ly = 2 * eb + qb, lz = 2 * ec + qc;
    R H[3][3];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      R hx = 0, hy = 0, hz = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        hx += R(dlgl(qa, a)) * sW[0 + ii][(2 * ea + a) + BX * (ly + BY * lz)];
        hy += R(dlgl(qb, a)) * sW[3 + ii][lx + BX * ((2 * eb + a) + BY * lz)];
        hz += R(dlgl(qc, a)) * sW[6 + ii][lx + BX * (ly + BY * (2 * ec + a))];
      }
      H[ii][0] = hx * s2h; H[ii][1] = hy * s2h; H[ii][2] = hz * s2h;
    }
    const R wq = R(0.125 * g.h * g.h * g.h * wlgl(qa) * wlgl(qb) * wlgl(qc));
    if constexpr (!ADJ) {
      const int nq = lx + BX * (ly + BY * lz);
      const R la = sLam[nq], m = sMu[nq];
      const R tr = H[0][0] + H[1][1] + H[2][2];
      sQ[0][q] = -wq * (la * tr + 2 * m * H[0][0]);
      sQ[1][q] = -wq * (la * tr + 2 * m * H[1][1]);
      sQ[2][q] = -wq * (la * tr + 2 * m * H[2][2]);
      sQ[3][q] = -wq * (m * (H[1][2] + H[2][1]));
      sQ[4][q] = -wq * (m * (H[0][2] + H[2][0]));
      sQ[5][q] = -wq * (m * (H[0][1] + H[1][0]));
    } else {
      sQ[0][q] = wq * H[0][0];
      sQ[1][q] = wq * H[1][1];
      sQ[2][q] = wq * H[2][2];
      sQ[3][q] = wq * (H[1][2] + H[2][1]);
      sQ[4][q] = wq * (H[0][2] + H[2][0]);
      sQ[5][q] = wq * (H[0][1] + H[1][0]);
    }
  }
  __syncthreads();

  const R vol = R(0.125 * g.h * g.h * g.h);
  for (int n = threadIdx.x; n < NB; n += blockDim.x) {
    const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
    if (lx >= nbx || ly >= nby || lz >= nbz) continue;
    const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
    int exs[2], pxs[2], eys[2], pys[2], ezs[2], pzs[2];
    const int nex = node_bricks(lx, cx, exs, pxs);
    const int ney = node_bricks(ly, cy, eys, pys);
    const int nez = node_bricks(lz, cz, ezs, pzs);
    // 1D weight sums of the tile's bricks that contain the node
    R Sx = 0, Sy = 0, Sz = 0;
    for (int a = 0; a < nex; ++a) Sx += R(wlgl(pxs[a]));
    for (int a = 0; a < ney; ++a) Sy += R(wlgl(pys[a]));
    for (int a = 0; a < nez; ++a) Sz += R(wlgl(pzs[a]));
    // u-rows: the stress-like tensor is nodal, so each direction factorizes
    R dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0}, dz[3] = {0, 0, 0};
    for (int b = 0; b < nex; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R cf = R(dlgl(a, pxs[b]) * wlgl(a));
        const int nx = (2 * exs[b] + a) + BX * (ly + BY * lz);
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) dx[ii] += cf * sT[3 * ii + 0][nx];
      }
    for (int b = 0; b < ney; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R cf = R(dlgl(a, pys[b]) * wlgl(a));
        const int ny = lx + BX * ((2 * eys[b] + a) + BY * lz);
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) dy[ii] += cf * sT[3 * ii + 1][ny];
      }
    for (int b = 0; b < nez; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R cf = R(dlgl(a, pzs[b]) * wlgl(a));
        const int nz = lx + BX * (ly + BY * (2 * ezs[b] + a));
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) dz[ii] += cf * sT[3 * ii + 2][nz];
      }
    // S-rows: sum of the point values of every tile brick containing the node
    R q6[6] = {0, 0, 0, 0, 0, 0};
    for (int a3 = 0; a3 < nez; ++a3)
      for (int a2 = 0; a2 < ney; ++a2)
        for (int a1 = 0; a1 < nex; ++a1) {
          const int qn = 27 * (exs[a1] + TX * (eys[a2] + TY * ezs[a3])) + pxs[a1] + 3 * pys[a2] + 9 * pzs[a3];
#pragma unroll
          for (int v = 0; v < 6; ++v) q6[v] += sQ[v][qn];
        }
    const size_t p = (size_t)pml_index(g, i, j, k);
#pragma unroll
    for (int v = 0; v < 6; ++v) atomic_add(&res[3 * nn + v * np + p], q6[v]);
    if (!is_dirichlet(g, i, j, k)) {
      const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
      const R f = vol * s2h;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
        atomic_add(&res[ii * nn + node], f * (Sy * Sz * dx[ii] + Sx * Sz * dy[ii] + Sx * Sy * dz[ii]));
    }
  }
}

// ---------------------------------------------------------------------------
// Nodal part of one RK4 stage.  With r the element residual of the stage input
// Y, the rates are K = (x1|PML, x2, M^{-1}(f - r - nodal PML terms)) and
//   mode 0:  acc = Xn + cA K,  Yout = Xn + cY K
//   mode 1:  acc += cA K,      Yout = Xn + cY K
//   mode 2:  Xn = acc + cA K
// The residual is cleared for the next stage.  Threads [0, n_nodes) handle
// the displacement rows, [n_nodes, n_nodes + n_pml) the PML rows.
template <typename R>
struct NodalArgs {
  const R* Yin;
  R* Yout;
  R* Xn;
  R* acc;
  R* res;
  const R* invMu;
  long long reg, rstr;
  R cA, cY;
  int mode;
  const int* src_node;        // nullptr: no load
  const double* src_dir;      // (nsrc, 3)
  const double* wav;          // (nsrc, wav_len)
  int wav_len, wav_idx;
  R* store;                   // x1 displacement of the produced register on the
  long long store_stride;     // interior closure (per source stride), or nullptr
};

template <typename R>
__global__ void __launch_bounds__(256) nodal_rk_kernel(Geo g, NodalArgs<R> A) {
  const int src = blockIdx.y;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)g.n_nodes, np = (size_t)g.n_pml;
  const R* Y = A.Yin + (size_t)src * A.reg;
  R* Yo = A.Yout ? A.Yout + (size_t)src * A.reg : nullptr;
  R* X = A.Xn + (size_t)src * A.reg;
  R* C = A.acc + (size_t)src * A.reg;
  R* res = A.res + (size_t)src * A.rstr;
  const R cA = A.cA, cY = A.cY;
  const int mode = A.mode;

  if (gid < (long long)nn) {
    const int node = (int)gid;
    const int k = node / g.plane;
    const int r_ = node - k * g.plane;
    const int j = r_ / g.NX, i = r_ - j * g.NX;
    if (is_dirichlet(g, i, j, k)) return;
    R u1[3], u2[3], rr[3], a2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u1[d] = Y[d * nn + node];
      u2[d] = Y[(3 + d) * nn + node];
      rr[d] = res[d * nn + node];
      res[d * nn + node] = R(0);
    }
    R f[3] = {0, 0, 0};
    if (A.src_node && A.src_node[src] == node) {
      const double s = A.wav[(size_t)src * A.wav_len + A.wav_idx];
#pragma unroll
      for (int d = 0; d < 3; ++d) f[d] = R(A.src_dir[3 * src + d] * s);
    }
    const R im = A.invMu[node];
#pragma unroll
    for (int d = 0; d < 3; ++d) a2[d] = im * (f[d] - rr[d]);
    if (in_pml(g, i, j, k)) {
      double mrd, mp;
      lumped_masses(g, i, j, k, mrd, mp);
      const PmlCoef c = pml_coef(g, i, j, k);
      const R kap = R(mp / (mrd + c.a * mp));
      R u0[3] = {0, 0, 0};
      if (c.nbeta >= 2) {
        const size_t p = (size_t)pml_index(g, i, j, k);
        const R* P = Y + 6 * nn;
#pragma unroll
        for (int d = 0; d < 3; ++d) u0[d] = P[(P_X0U + d) * np + p];
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
        a2[d] -= kap * (R(c.b) * u2[d] + R(c.c) * u1[d] + R(c.d) * u0[d]);
    }
    R out1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const size_t o1 = d * nn + node, o2 = (3 + d) * nn + node;
      if (mode == 2) {
        X[o1] = out1[d] = C[o1] + cA * u2[d];
        X[o2] = C[o2] + cA * a2[d];
      } else {
        const R x1 = X[o1], x2 = X[o2];
        if (mode == 0) {
          C[o1] = x1 + cA * u2[d];
          C[o2] = x2 + cA * a2[d];
        } else {
          C[o1] += cA * u2[d];
          C[o2] += cA * a2[d];
        }
        Yo[o1] = out1[d] = x1 + cY * u2[d];
        Yo[o2] = x2 + cY * a2[d];
      }
    }
    if (A.store) {
      const int mi = interior_index(g, i, j, k);
      if (mi >= 0) {
        R* S = A.store + (size_t)src * A.store_stride;
#pragma unroll
        for (int d = 0; d < 3; ++d) S[(size_t)d * g.n_int + mi] = out1[d];
      }
    }
    return;
  }
  const long long pp = gid - (long long)nn;
  if (pp >= (long long)np) return;
  const size_t p = (size_t)pp;
  int i, j, k;
  pml_coords(g, (int)p, i, j, k);
  const PmlCoef c = pml_coef(g, i, j, k);
  double mrd, mp;
  lumped_masses(g, i, j, k, mrd, mp);
  const bool hist = c.nbeta >= 2;
  const R* PY = Y + 6 * nn;
  R* PX = X + 6 * nn;
  R* PC = C + 6 * nn;
  R* PO = Yo ? Yo + 6 * nn : nullptr;
  R* rS = res + 3 * nn;
  const R ia = R(1.0 / c.a), iam = R(1.0 / (c.a * mp));
  const R cb = R(c.b), cc = R(c.c), cd = R(c.d);

  auto upd = [&](int comp, R rate) {
    const size_t o = (size_t)comp * np + p;
    if (mode == 2) {
      PX[o] = PC[o] + cA * rate;
    } else {
      const R x = PX[o];
      if (mode == 0) PC[o] = x + cA * rate;
      else PC[o] += cA * rate;
      PO[o] = x + cY * rate;
    }
  };
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    const R s1 = PY[(P_X1S + v) * np + p], s2 = PY[(P_X2S + v) * np + p];
    const R s0 = hist ? PY[(P_X0S + v) * np + p] : R(0);
    const R rv = rS[v * np + p];
    rS[v * np + p] = R(0);
    const R a2 = -rv * iam - ia * (cb * s2 + cc * s1 + cd * s0);
    if (hist) upd(P_X0S + v, s1);
    upd(P_X1S + v, s2);
    upd(P_X2S + v, a2);
  }
  if (hist && !is_dirichlet(g, i, j, k)) {
    const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
#pragma unroll
    for (int d = 0; d < 3; ++d) upd(P_X0U + d, Y[d * nn + node]);
  }
}

// 1/M_uu at every node (0 on Dirichlet nodes): rho (m_rd + a m_p).
template <typename R>
__global__ void inv_mass_kernel(Geo g, const double* __restrict__ rho, R* __restrict__ invMu) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= g.n_nodes) return;
  const int k = node / g.plane, r_ = node - k * g.plane;
  const int j = r_ / g.NX, i = r_ - j * g.NX;
  if (is_dirichlet(g, i, j, k)) {
    invMu[node] = R(0);
    return;
  }
  double mrd, mp;
  lumped_masses(g, i, j, k, mrd, mp);
  const PmlCoef c = pml_coef(g, i, j, k);
  invMu[node] = R(1.0 / (rho[material_index(g, i, j, k)] * (mrd + c.a * mp)));
}

}  // namespace pmlfwi
