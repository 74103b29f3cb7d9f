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
//
// Element work is done per tile of bricks: a workgroup per (tile, source), or
// per tile with the sources in turn where a result is summed over sources (the
// gradient); each thread keeps one node of the tile's node box.  The PML
// operator runs as two launches, one per row type.  Scatter without atomics:
// a node lies on the upper face (local index 2*count) of at most one tile per
// axis, so the set c of axes on which it is an upper-face node differs for
// every tile containing it.  A tile
// stores its partial sum for a box node with a plain store into partial
// array c; the nodal kernel adds the arrays c that can be non-zero for the
// node.  Array 0 uses the register index spaces (full grid for u-rows, PML
// shell for S-rows); arrays c != 0 use the full grid with the axes in c
// compressed to the upper-face positions.  Entries nobody writes stay zero
// from the initial clear.
//
// Tiles are handed to the XCDs in contiguous runs: workgroup b of a grid
// whose size is a multiple of 8 runs on XCD b mod 8 and takes tile
// (b mod 8) * (grid/8) + b / 8, so neighbouring tiles share an L2.
#pragma once
#include "geometry.h"

// Threads of an element-kernel workgroup: at least the tile's box nodes (one
// node per thread; the kernels loop over the tile's LGL points in strides of
// the workgroup size).  512 fits the 11 x 9 x 5 node box of a 5x4x2 tile.
#ifndef PMLFWI_ETHREADS
#define PMLFWI_ETHREADS 512
#endif
// Threads per nodal workgroup (128 measured a little faster than 256, 512 slower).
#ifndef PMLFWI_NODAL_THREADS
#define PMLFWI_NODAL_THREADS 128
#endif

namespace pmlfwi {

enum { P_X0U = 0, P_X0S = 3, P_X1S = 9, P_X2S = 15, P_NCOMP = 21, U_NCOMP = 6 };

// State register of one source.  Node part: x1 u as [sn][3], then x2 u as
// [sn][3]; PML part (from entry 6 sn): x0 u as [sp][3], then x0 S, x1 S and
// x2 S as [sp][6] each.  A field's components at a node are contiguous, so a
// kernel loads or stores them as one vector.
// Entry of u-component d (0..2: x1 u, 3..5: x2 u) of node `node`:
__host__ __device__ __forceinline__ size_t u_at(size_t nn, int d, size_t node) {
  return d < 3 ? 3 * node + d : 3 * nn + 3 * node + (d - 3);
}
// Entry of PML component q (P_X0U .. P_NCOMP-1) of PML node p, relative to
// the PML part:
__host__ __device__ __forceinline__ size_t p_at(size_t np, int q, size_t p) {
  if (q < P_X0S) return 3 * p + q;
  const int b = q < P_X1S ? P_X0S : (q < P_X2S ? P_X1S : P_X2S);
  return (size_t)b * np + 6 * p + (q - b);
}

// Voigt slot of the symmetric pair (i, k).
__host__ __device__ constexpr int vidx(int i, int k) { return i == k ? i : 6 - i - k; }

// Derivative of 1D basis a at LGL point q: D[q][a] (nodes -1, 0, 1).
__device__ __forceinline__ float dlgl(int q, int a) {
  // rows q = 0: (-3/2, 2, -1/2); q = 1: (-1/2, 0, 1/2); q = 2: (1/2, -2, 3/2)
  const float r0 = a == 0 ? -1.5f : (a == 1 ? 2.0f : -0.5f);
  const float r1 = a == 0 ? -0.5f : (a == 1 ? 0.0f : 0.5f);
  const float r2 = a == 0 ? 0.5f : (a == 1 ? -2.0f : 1.5f);
  return q == 0 ? r0 : (q == 1 ? r1 : r2);
}
__device__ __forceinline__ double wlgl(int a) { return a == 1 ? 4.0 / 3.0 : 1.0 / 3.0; }

// The same derivatives in closed form, for the hot loops: with the LGL nodes
// xi = -1, 0, 1, the basis functions l_0 = xi (xi - 1) / 2, l_1 = 1 - xi^2,
// l_2 = xi (xi + 1) / 2 have l_p' (xi) = (3 (p - 1)^2 - 2) xi + (p - 1) / 2.
// dbasis(x, a) = l_a'(x) for a known at compile time (unrolled loops), x the
// point's coordinate xi_q = q - 1 (exact in any precision); dbasis_coef gives
// the two factors for a basis index known only at run time.
template <typename R>
__device__ __forceinline__ R dbasis(R x, int a) {
  return a == 0 ? x - R(0.5) : (a == 1 ? R(-2) * x : x + R(0.5));
}
template <typename R>
__device__ __forceinline__ void dbasis_coef(int p, R& c1, R& c0) {
  const int m = p - 1;
  c1 = R(3 * m * m - 2);
  c0 = R(0.5) * R(m);
}

struct Tile {  // bricks [x, x+cx) x [y, y+cy) x [z, z+cz)
  int x, y, z, c;  // c = cx | cy << 8 | cz << 16
};

struct Part {             // partial residual arrays of one source
  long long off[8];       // element offset of array c (array 0 at 0)
  long long size[8];      // nodes of array c (c != 0: compressed box)
  int nx[8], ny[8];       // x / y extents of array c
  long long per_src;      // elements per source
};

__device__ __forceinline__ int face_mask(const Geo& g, int i, int j, int k) {
  return (g.fo[i] >= 0) | ((g.fo[ax_y(g) + j] >= 0) << 1) | ((g.fo[ax_z(g) + k] >= 0) << 2);
}

__device__ __forceinline__ size_t part_node(const Geo& g, const Part& P, int c, int i, int j, int k) {
  const int ii = (c & 1) ? g.fo[i] : i;
  const int jj = (c & 2) ? g.fo[ax_y(g) + j] : j;
  const int kk = (c & 4) ? g.fo[ax_z(g) + k] : k;
  return (size_t)ii + (size_t)P.nx[c] * ((size_t)jj + (size_t)P.ny[c] * kk);
}

// Offsets of a node's rows in partial array c (within one source).  A node's
// rows are contiguous, so they are stored and gathered as short vectors: array
// 0 holds the three u-rows of every node ([sn][3]) followed by the six S-rows
// of every PML node ([sp][6]); array c != 0 holds [size_c][3] u-rows followed
// by [size_c][6] S-rows, indexed by the node's place in the compressed box.
// u-row d sits at u + d, S-row v at s + v.  Computed once per node before its
// stores, so the lane-varying lookups of the array constants and face
// ordinals are waited for once rather than once per row.
struct RowAddr {
  size_t u, s;
};

__device__ __forceinline__ RowAddr row_addr(const Geo& g, const Part& P, int c, int i, int j, int k,
                                            size_t node, size_t p) {
  RowAddr a;
  if (c == 0) {
    a.u = 3 * node;
    a.s = 3 * (size_t)g.sn + 6 * p;
    return a;
  }
  const size_t n = part_node(g, P, c, i, j, k);
  a.u = (size_t)P.off[c] + 3 * n;
  a.s = (size_t)P.off[c] + 3 * (size_t)P.size[c] + 6 * n;
  return a;
}

__device__ __forceinline__ int xcd_tile() {
  const int per = gridDim.x >> 3;
  const int b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

// Per-dimension list of the bricks of a tile that contain local node l:
// (brick offset, position of the node in that brick).  At most two.
__device__ __forceinline__ int node_bricks(int l, int cnt, int* e, int* p) {
  if (l & 1) {
    e[0] = (l - 1) >> 1;
    p[0] = 1;
    e[1] = e[0];
    p[1] = 1;
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
  if (n == 1) {
    e[1] = e[0];
    p[1] = p[0];
  }
  return n;
}

// The two candidate bricks of a tile along one axis for local node l
// (0 <= l <= 2 cnt): the brick below (l odd: the only one) and the brick above
// (l even), as offsets se * brick + sp * (position of the node in the brick)
// into brick-local arrays, each with a flag telling whether it holds the node.
__device__ __forceinline__ void axis_bricks(int l, int cnt, int se, int sp, int o[2], bool v[2]) {
  const int e0 = (l - 1) >> 1, e1 = l >> 1;
  o[0] = se * e0 + sp * (l - 2 * e0);
  o[1] = se * e1 + sp * (l - 2 * e1);
  v[0] = l >= 1;
  v[1] = !(l & 1) && e1 < cnt;
}

template <typename R>
__device__ __forceinline__ void atomic_add(R* p, R v) {
  unsafeAtomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// Interior bricks: r_u += K_RD u  (u = x1 displacement of the input register).
// GRAD: also  g -= b_s * sum_e w|J| (div z div u_f, 2 eps(z):eps(u_f)) at the
// LGL nodes, z = the displacement read here, u_f = stored forward stage field,
// summed over sources and added to FP64 accumulators (gacc: [8][2][n_nodes],
// slot c indexed like the partial arrays).
template <typename R, int TX, int TY, int TZ, bool GRAD, bool SRCLOOP>
__global__ void __launch_bounds__(PMLFWI_ETHREADS)
interior_element_kernel(Geo g, const Tile* __restrict__ tiles, int ntiles, int nsrc,
                        const R* __restrict__ Ybase, long long ystride, const R* __restrict__ lam,
                        const R* __restrict__ mu, R* __restrict__ rbase, Part PT,
                        const R* __restrict__ fwd, long long fstride, double gw,
                        double* __restrict__ gacc, Part PG) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NP = 27 * TX * TY * TZ;
  __shared__ R sU[3][NB];
  __shared__ R sLam[NB], sMu[NB];
  __shared__ R sS[6][NP];
  __shared__ R sR[3][NP];   // brick-local rows B^T S, summed over bricks per node below
  __shared__ R sV[GRAD ? 3 : 1][GRAD ? NB : 1];
  __shared__ R sG[GRAD ? 2 : 1][GRAD ? NP : 1];
  __shared__ double sGacc[GRAD ? 2 : 1][GRAD ? NB : 1];   // summed over sources

  static_assert(NB <= PMLFWI_ETHREADS, "one box node per thread");
  const int ti = xcd_tile();
  if (ti >= ntiles) return;
  const Tile t = tiles[ti];
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const size_t nn = (size_t)g.sn;
  const R s2h = R(2.0 / g.h);
  const double wh3 = 0.125 * g.h * g.h * g.h;

  // this thread's box node and its constants, shared by the sources
  const int n = threadIdx.x;
  const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
  const bool live = n < NB && lx <= 2 * cx && ly <= 2 * cy && lz <= 2 * cz;
  const int i = 2 * t.x + lx, j = 2 * t.y + ly, k = 2 * t.z + lz;
  const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
  const int mi = live ? interior_index(g, i, j, k) : 0;
  const int cs = (lx == 2 * cx) | ((ly == 2 * cy) << 1) | ((lz == 2 * cz) << 2);
  if (live) {
    sLam[n] = lam[mi];
    sMu[n] = mu[mi];
    if constexpr (GRAD) {
      sGacc[0][n] = 0.0;
      sGacc[1][n] = 0.0;
    }
  }

  static_assert(SRCLOOP || !GRAD, "gradient sums over sources inside the workgroup");
  const int src0 = SRCLOOP ? 0 : (int)blockIdx.y, src1 = SRCLOOP ? nsrc : src0 + 1;
  for (int src = src0; src < src1; ++src) {
    const R* Yu = Ybase + (size_t)src * ystride;
    if (live) {
#pragma unroll
      for (int d = 0; d < 3; ++d) sU[d][n] = Yu[u_at(nn, d, node)];
      if constexpr (GRAD) {
        const R* F = fwd + (size_t)src * fstride;
#pragma unroll
        for (int d = 0; d < 3; ++d) sV[d][n] = __builtin_nontemporal_load(&F[3 * (size_t)mi + d]);
      }
    }
    __syncthreads();

    for (int q = threadIdx.x; q < NP; q += blockDim.x) {
      const int pt = q % 27, e = q / 27;
      const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
      if (ea >= cx || eb >= cy || ec >= cz) continue;
      const int qa = pt % 3, qb = (pt / 3) % 3, qc = pt / 9;
      const int px = 2 * ea + qa, py = 2 * eb + qb, pz = 2 * ec + qc;   // box node of the point
      const int nq = px + BX * (py + BY * pz);
      R G[3][3], Gf[3][3];
      const R xa = R(qa - 1), xb = R(qb - 1), xc = R(qc - 1);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        R gx = 0, gy = 0, gz = 0, fx = 0, fy = 0, fz = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const R cxa = dbasis(xa, a), cya = dbasis(xb, a), cza = dbasis(xc, a);
          const int nx = (2 * ea + a) + BX * (py + BY * pz);
          const int ny = px + BX * ((2 * eb + a) + BY * pz);
          const int nz = px + BX * (py + BY * (2 * ec + a));
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
      const R wq = R(wh3 * wlgl(qa) * wlgl(qb) * wlgl(qc));
      const R la = sLam[nq], m = sMu[nq];
      const R tr = G[0][0] + G[1][1] + G[2][2];
      sS[0][q] = wq * (la * tr + 2 * m * G[0][0]);
      sS[1][q] = wq * (la * tr + 2 * m * G[1][1]);
      sS[2][q] = wq * (la * tr + 2 * m * G[2][2]);
      sS[3][q] = wq * (m * (G[1][2] + G[2][1]));
      sS[4][q] = wq * (m * (G[0][2] + G[2][0]));
      sS[5][q] = wq * (m * (G[0][1] + G[1][0]));
      if constexpr (GRAD) {
        // per-stage products in the state precision; summed in FP64 below
        const R du = Gf[0][0] + Gf[1][1] + Gf[2][2];
        R ee = 2 * (G[0][0] * Gf[0][0] + G[1][1] * Gf[1][1] + G[2][2] * Gf[2][2]);
        ee += (G[1][2] + G[2][1]) * (Gf[1][2] + Gf[2][1]);
        ee += (G[0][2] + G[2][0]) * (Gf[0][2] + Gf[2][0]);
        ee += (G[0][1] + G[1][0]) * (Gf[0][1] + Gf[1][0]);
        sG[0][q] = wq * tr * du;
        sG[1][q] = wq * ee;
      }
    }
    __syncthreads();

    // brick-local rows: for local node (pa, pb, pc) of brick e and component i,
    // sum over the points on the three lines through the node of
    // D(point, node) times the stress column of that axis (sum-factorized B^T S)
    for (int q = threadIdx.x; q < NP; q += blockDim.x) {
      const int pt = q % 27, e0 = q - pt;
      const int pa = pt % 3, pb = (pt / 3) % 3, pc = pt / 9;
      R ax1, ax0, ay1, ay0, az1, az0;
      dbasis_coef<R>(pa, ax1, ax0);
      dbasis_coef<R>(pb, ay1, ay0);
      dbasis_coef<R>(pc, az1, az0);
      R r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        // derivative of the node's basis function at point a: c1 xi_a + c0
        const R cxa = ax0 + R(a - 1) * ax1, cya = ay0 + R(a - 1) * ay1, cza = az0 + R(a - 1) * az1;
        const int qx = e0 + a + 3 * pb + 9 * pc;
        const int qy = e0 + pa + 3 * a + 9 * pc;
        const int qz = e0 + pa + 3 * pb + 9 * a;
        r0 += cxa * sS[0][qx] + cya * sS[5][qy] + cza * sS[4][qz];
        r1 += cxa * sS[5][qx] + cya * sS[1][qy] + cza * sS[3][qz];
        r2 += cxa * sS[4][qx] + cya * sS[3][qy] + cza * sS[2][qz];
      }
      sR[0][q] = r0;
      sR[1][q] = r1;
      sR[2][q] = r2;
    }
    __syncthreads();

    R* res = rbase + (size_t)src * PT.per_src;
    if (live) {
      int ox[2], oy[2], oz[2];
      bool vx[2], vy[2], vz[2];
      axis_bricks(lx, cx, 27, 1, ox, vx);
      axis_bricks(ly, cy, 27 * TX, 3, oy, vy);
      axis_bricks(lz, cz, 27 * TX * TY, 9, oz, vz);
      R r0 = 0, r1 = 0, r2 = 0;
      R gl = 0, gm = 0;
#pragma unroll
      for (int a3 = 0; a3 < 2; ++a3)
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int a1 = 0; a1 < 2; ++a1) {
            if (!(vx[a1] && vy[a2] && vz[a3])) continue;
            const int qn = ox[a1] + oy[a2] + oz[a3];
            r0 += sR[0][qn];
            r1 += sR[1][qn];
            r2 += sR[2][qn];
            if constexpr (GRAD) {
              gl += sG[0][qn];
              gm += sG[1][qn];
            }
          }
      if (!is_dirichlet(g, i, j, k)) {
        const RowAddr ra = row_addr(g, PT, cs, i, j, k, node, 0);
        res[ra.u] = r0 * s2h;
        res[ra.u + 1] = r1 * s2h;
        res[ra.u + 2] = r2 * s2h;
      }
      if constexpr (GRAD) {
        sGacc[0][n] += (double)gl;
        sGacc[1][n] += (double)gm;
      }
    }
    __syncthreads();
  }
  if constexpr (GRAD) {
    if (live) {
      const size_t o = (size_t)PG.off[cs] + part_node(g, PG, cs, i, j, k), gs = (size_t)PG.size[cs];
      const double a0 = gacc[o], a1 = gacc[o + gs];
      gacc[o] = a0 + gw * sGacc[0][n];
      gacc[o + gs] = a1 + gw * sGacc[1][n];
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
//
// The S-rows depend on the displacements only (through W and Q) and the
// u-rows on the stresses only (through T), so the operator splits into two
// independent parts (PART: PML_SROWS, PML_UROWS or both).  A workgroup works
// in up to three phases per source: (1) every box node's register values
// become the nodal fields W and/or T in LDS, (2) S-rows: every LGL point of
// every brick forms Q from the gradients of W, (3) every box node sums its
// u-rows (a stencil along each axis, T being nodal) and/or S-rows and stores
// them.
enum { PML_SROWS = 1, PML_UROWS = 2, PML_ALL = 3 };

template <typename R>
struct PmlNode {          // register values of one box node for one source
  R u1[3], u2[3], u0[3], s0[6], s1[6], s2[6];
};

template <typename R, bool U, bool S>
__device__ __forceinline__ void pml_load_node(const R* __restrict__ Y, size_t nn, size_t np, size_t gnode,
                                              size_t gp, bool hist, PmlNode<R>& v) {
  const R* P = Y + 6 * nn;
  if constexpr (U) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v.u1[d] = Y[u_at(nn, d, gnode)];
      v.u2[d] = Y[u_at(nn, 3 + d, gnode)];
      v.u0[d] = hist ? P[p_at(np, P_X0U + d, gp)] : R(0);
    }
  }
  if constexpr (S) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      v.s1[c] = P[p_at(np, P_X1S + c, gp)];
      v.s2[c] = P[p_at(np, P_X2S + c, gp)];
      v.s0[c] = hist ? P[p_at(np, P_X0S + c, gp)] : R(0);
    }
  }
}

// Phase 1 for one node: W (U) from the displacements.
template <typename R, int NB>
__device__ __forceinline__ void pml_node_w(const PmlNode<R>& v, const R Le[3], const R Lp[3], const R Lw[3], int n,
                                           R (&sW)[9][NB]) {
#pragma unroll
  for (int kk = 0; kk < 3; ++kk)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) sW[3 * kk + ii][n] = Le[kk] * v.u2[ii] + Lp[kk] * v.u1[ii] + Lw[kk] * v.u0[ii];
}

// Phase 1 for one node: T from the stresses.
template <typename R, bool ADJ, int NB>
__device__ __forceinline__ void pml_node_t(const PmlNode<R>& v, const R Le[3], const R Lp[3], const R Lw[3], R la,
                                           R m, int n, R (&sT)[9][NB]) {
  if constexpr (!ADJ) {
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const int c = vidx(ii, kk);
        sT[3 * ii + kk][n] = Le[kk] * v.s2[c] + Lp[kk] * v.s1[c] + Lw[kk] * v.s0[c];
      }
  } else {
    const R t2 = v.s2[0] + v.s2[1] + v.s2[2], t1 = v.s1[0] + v.s1[1] + v.s1[2], t0 = v.s0[0] + v.s0[1] + v.s0[2];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const int c = vidx(ii, kk);
        const R z = Le[kk] * v.s2[c] + Lp[kk] * v.s1[c] + Lw[kk] * v.s0[c];
        R val = (ii == kk ? R(2) : R(1)) * m * z;
        if (ii == kk) val += la * (Le[ii] * t2 + Lp[ii] * t1 + Lw[ii] * t0);
        sT[3 * ii + kk][n] = -val;
      }
  }
}

// Q (6 values) at LGL point q of the tile's bricks; false for points of bricks
// outside a ragged tile.  sLam, sMu: box-node materials (forward only).
template <typename R, int TX, int TY, int TZ, bool ADJ>
__device__ __forceinline__ bool pml_point_value(const Geo& g, int cx, int cy, int cz, int q,
                                                const R* __restrict__ sW, const R* __restrict__ sLam,
                                                const R* __restrict__ sMu, R Q[6]) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, NB = BX * BY * (2 * TZ + 1);
  const R s2h = R(2.0 / g.h);
  const int pt = q % 27, e = q / 27;
  const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
  if (ea >= cx || eb >= cy || ec >= cz) return false;
  const int qa = pt % 3, qb = (pt / 3) % 3, qc = pt / 9;
  const int lx = 2 * ea + qa, ly = 2 * eb + qb, lz = 2 * ec + qc;
  R H[3][3];
  const R xa = R(qa - 1), xb = R(qb - 1), xc = R(qc - 1);
#pragma unroll
  for (int ii = 0; ii < 3; ++ii) {
    R hx = 0, hy = 0, hz = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      hx += dbasis(xa, a) * sW[(0 + ii) * NB + (2 * ea + a) + BX * (ly + BY * lz)];
      hy += dbasis(xb, a) * sW[(3 + ii) * NB + lx + BX * ((2 * eb + a) + BY * lz)];
      hz += dbasis(xc, a) * sW[(6 + ii) * NB + lx + BX * (ly + BY * (2 * ec + a))];
    }
    H[ii][0] = hx * s2h; H[ii][1] = hy * s2h; H[ii][2] = hz * s2h;
  }
  const R wq = R(0.125 * g.h * g.h * g.h * wlgl(qa) * wlgl(qb) * wlgl(qc));
  if constexpr (!ADJ) {
    const int nq = lx + BX * (ly + BY * lz);
    const R la = sLam[nq], m = sMu[nq];
    const R tr = H[0][0] + H[1][1] + H[2][2];
    Q[0] = -wq * (la * tr + 2 * m * H[0][0]);
    Q[1] = -wq * (la * tr + 2 * m * H[1][1]);
    Q[2] = -wq * (la * tr + 2 * m * H[2][2]);
    Q[3] = -wq * (m * (H[1][2] + H[2][1]));
    Q[4] = -wq * (m * (H[0][2] + H[2][0]));
    Q[5] = -wq * (m * (H[0][1] + H[1][0]));
  } else {
    Q[0] = wq * H[0][0];
    Q[1] = wq * H[1][1];
    Q[2] = wq * H[2][2];
    Q[3] = wq * (H[1][2] + H[2][1]);
    Q[4] = wq * (H[0][2] + H[2][0]);
    Q[5] = wq * (H[0][1] + H[1][0]);
  }
  return true;
}

// Along one axis, the u-row term of local node l (0 <= l <= 2 cnt) is
// sum_k c[k] T(l - 2 + k): over the tile's bricks containing l, the LGL weight
// of point a times the derivative of the node's basis function at a, placed
// at the box node of a.  Brick below (l odd: position 1, else 2) and brick
// above (l even: position 0) give
//   l odd:   (0, 2/3, 0, -2/3, 0)
//   l even:  below (-1/6, 2/3, 1/2, 0, 0) + above (0, 0, -1/2, -2/3, 1/6).
// S: the sum of the 1D weights of those bricks at l.  Indices are clamped
// to the tile box (the clamped reads have coefficient 0).
template <typename R>
__device__ __forceinline__ void axis_stencil(int l, int cnt, R c[5], int o[5], R& S) {
  const bool odd = l & 1, lo = l >= 1, hi = !odd && (l >> 1) < cnt;
  const R third = R(1.0 / 3.0), sixth = R(1.0 / 6.0), two3 = R(2.0 / 3.0);
  c[0] = (!odd && lo) ? -sixth : R(0);
  c[1] = lo ? two3 : R(0);
  c[2] = odd ? R(0) : R(lo ? 0.5 : 0.0) - R(hi ? 0.5 : 0.0);
  c[3] = (odd || hi) ? -two3 : R(0);
  c[4] = hi ? sixth : R(0);
  S = odd ? R(4.0 / 3.0) : R(lo ? third : R(0)) + R(hi ? third : R(0));
#pragma unroll
  for (int k = 0; k < 5; ++k) o[k] = min(max(l - 2 + k, 0), 2 * cnt);
}

// Phase 3, u-rows of box node (lx, ly, lz) from the nodal T.
template <typename R, int TX, int TY, int TZ>
__device__ __forceinline__ void pml_u_rows(const Geo& g, int cx, int cy, int cz, int lx, int ly, int lz,
                                           const R* __restrict__ sT, R out[3]) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, NB = BX * BY * (2 * TZ + 1);
  R c[5], Sx, Sy, Sz;
  int o[5];
  R dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0}, dz[3] = {0, 0, 0};
  axis_stencil<R>(lx, cx, c, o, Sx);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int n = o[k] + BX * (ly + BY * lz);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) dx[ii] += c[k] * sT[(3 * ii + 0) * NB + n];
  }
  axis_stencil<R>(ly, cy, c, o, Sy);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int n = lx + BX * (o[k] + BY * lz);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) dy[ii] += c[k] * sT[(3 * ii + 1) * NB + n];
  }
  axis_stencil<R>(lz, cz, c, o, Sz);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int n = lx + BX * (ly + BY * o[k]);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) dz[ii] += c[k] * sT[(3 * ii + 2) * NB + n];
  }
  const R f = R(0.125 * g.h * g.h * g.h) * R(2.0 / g.h);
#pragma unroll
  for (int ii = 0; ii < 3; ++ii) out[ii] = f * (Sy * Sz * dx[ii] + Sx * Sz * dy[ii] + Sx * Sy * dz[ii]);
}

// Phase 3, S-rows of box node (lx, ly, lz): the sum of the point values of
// every tile brick containing the node.
template <typename R, int TX, int TY, int TZ>
__device__ __forceinline__ void pml_s_rows(int cx, int cy, int cz, int lx, int ly, int lz,
                                           const R* __restrict__ sQ, R q6[6]) {
  constexpr int NP = 27 * TX * TY * TZ;
  int ox[2], oy[2], oz[2];
  bool vx[2], vy[2], vz[2];
  axis_bricks(lx, cx, 27, 1, ox, vx);
  axis_bricks(ly, cy, 27 * TX, 3, oy, vy);
  axis_bricks(lz, cz, 27 * TX * TY, 9, oz, vz);
#pragma unroll
  for (int v = 0; v < 6; ++v) q6[v] = 0;
#pragma unroll
  for (int a3 = 0; a3 < 2; ++a3)
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int a1 = 0; a1 < 2; ++a1) {
        if (!(vx[a1] && vy[a2] && vz[a3])) continue;
        const int qn = ox[a1] + oy[a2] + oz[a3];
#pragma unroll
        for (int v = 0; v < 6; ++v) q6[v] += sQ[v * NP + qn];
      }
}

// Per-node constants of phase 1: PML coefficients, history flag, indices.
template <typename R>
__device__ __forceinline__ void pml_node_setup(const Geo& g, int gi, int gj, int gk, R Le[3], R Lp[3], R Lw[3],
                                               bool& hist, size_t& gnode, size_t& gp) {
  gnode = (size_t)gi + (size_t)g.NX * (gj + (size_t)g.NY * gk);
  gp = (size_t)pml_index(g, gi, gj, gk);
  // products of the 1D stretching factors in the state precision
  const int nt = ax_n(g);
  const double* A = g.tab;
  const double* B = g.tab + nt;
  const R ax = R(A[gi]), ay = R(A[ax_y(g) + gj]), az = R(A[ax_z(g) + gk]);
  const R bx = R(B[gi]), by = R(B[ax_y(g) + gj]), bz = R(B[ax_z(g) + gk]);
  hist = (B[gi] > 0.0) + (B[ax_y(g) + gj] > 0.0) + (B[ax_z(g) + gk] > 0.0) >= 2;   // as the layout decides
  Le[0] = ay * az; Lp[0] = ay * bz + by * az; Lw[0] = by * bz;
  Le[1] = ax * az; Lp[1] = ax * bz + bx * az; Lw[1] = bx * bz;
  Le[2] = ax * ay; Lp[2] = ax * by + bx * ay; Lw[2] = bx * by;
}

// One workgroup per (tile, source) (SRCLOOP = false) or per tile with the
// sources in turn (SRCLOOP = true); PART selects the rows (see above).
template <typename R, int TX, int TY, int TZ, bool ADJ, bool SRCLOOP, int PART>
__global__ void __launch_bounds__(PMLFWI_ETHREADS)
pml_element_kernel(Geo g, const Tile* __restrict__ tiles, int ntiles, int nsrc,
                   const R* __restrict__ Ybase, long long ystride, const R* __restrict__ lam,
                   const R* __restrict__ mu, R* __restrict__ rbase, Part PT) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NP = 27 * TX * TY * TZ;
  constexpr bool DS = PART & PML_SROWS, DU = PART & PML_UROWS;
  constexpr bool MATQ = DS && !ADJ;   // box-node materials in LDS for the forward Q
  static_assert(NB <= PMLFWI_ETHREADS, "one box node per thread");
  __shared__ R sW[DS ? 9 : 1][DS ? NB : 1];   // [3k + i]: Le_kk u'_i + Lp_kk u_i + Lw_kk ubar_i
  __shared__ R sQ[DS ? 6 : 1][DS ? NP : 1];
  __shared__ R sT[DU ? 9 : 1][DU ? NB : 1];   // [3i + k]: nodal stress-like tensor of the u-rows
  __shared__ R sLam[MATQ ? NB : 1], sMu[MATQ ? NB : 1];

  const int ti = xcd_tile();
  if (ti >= ntiles) return;
  const Tile t = tiles[ti];
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const size_t nn = (size_t)g.sn, np = (size_t)g.sp;

  // this thread's box node and its constants, shared by the sources
  const int n = threadIdx.x;
  const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
  const bool live = n < NB && lx <= 2 * cx && ly <= 2 * cy && lz <= 2 * cz;
  const int gi = 2 * t.x + lx, gj = 2 * t.y + ly, gk = 2 * t.z + lz;
  R Le[3] = {0, 0, 0}, Lp[3] = {0, 0, 0}, Lw[3] = {0, 0, 0}, la = 0, m = 0;
  bool hist = false, free_u = false;
  size_t gnode = 0, gp = 0;
  RowAddr ra{};
  if (live) {
    pml_node_setup<R>(g, gi, gj, gk, Le, Lp, Lw, hist, gnode, gp);
    const int cs = (lx == 2 * cx) | ((ly == 2 * cy) << 1) | ((lz == 2 * cz) << 2);
    ra = row_addr(g, PT, cs, gi, gj, gk, gnode, gp);
    free_u = !is_dirichlet(g, gi, gj, gk);
    if constexpr (MATQ || (DU && ADJ)) {
      const int mi = material_index(g, gi, gj, gk);
      la = lam[mi];
      m = mu[mi];
      if constexpr (MATQ) {
        sLam[n] = la;
        sMu[n] = m;
      }
    }
  }

  const int src0 = SRCLOOP ? 0 : (int)blockIdx.y, src1 = SRCLOOP ? nsrc : src0 + 1;
  for (int src = src0; src < src1; ++src) {
    const R* Y = Ybase + (size_t)src * ystride;
    if (live) {
      PmlNode<R> v;
      pml_load_node<R, DS, DU>(Y, nn, np, gnode, gp, hist, v);
      if constexpr (DS) pml_node_w<R, NB>(v, Le, Lp, Lw, n, sW);
      if constexpr (DU) pml_node_t<R, ADJ, NB>(v, Le, Lp, Lw, la, m, n, sT);
    }
    __syncthreads();
    if constexpr (DS) {
      for (int q = threadIdx.x; q < NP; q += blockDim.x) {
        R Q[6];
        if (!pml_point_value<R, TX, TY, TZ, ADJ>(g, cx, cy, cz, q, &sW[0][0], &sLam[0], &sMu[0], Q)) continue;
#pragma unroll
        for (int v = 0; v < 6; ++v) sQ[v][q] = Q[v];
      }
      __syncthreads();
    }
    R* res = rbase + (size_t)src * PT.per_src;
    if (live) {
      if constexpr (DS) {
        R q6[6];
        pml_s_rows<R, TX, TY, TZ>(cx, cy, cz, lx, ly, lz, &sQ[0][0], q6);
#pragma unroll
        for (int v = 0; v < 6; ++v) res[ra.s + v] = q6[v];
      }
      if constexpr (DU) {
        if (free_u) {
          R u3[3];
          pml_u_rows<R, TX, TY, TZ>(g, cx, cy, cz, lx, ly, lz, &sT[0][0], u3);
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) res[ra.u + ii] = u3[ii];
        }
      }
    }
    if constexpr (SRCLOOP) __syncthreads();
  }
}

// Gradient terms of the PML S-rows under the material extension (the chain
// rule through the interface values a PML node takes, used when the full
// gradient is asked for).  The S-row of a PML node j in brick e carries
// -w_q [mu_j (H + H^T) + lam_j tr(H) I], H_ik = sum_L L_kk d_k u^L_i at the
// node's point, u^L the forward stage's (u', u, ubar) for L = (Le, Lp, Lw).
// With z the adjoint stress at j (x1 S part of the adjoint stage register),
// the gradient gains gw * (-w_q) (tr(H) sum_a z_aa, sum_v z_v (H_ab + H_ba))
// at node j, summed over sources and the node's PML bricks, into the FP64
// accumulators indexed like the partial arrays (gacc: full grid, 2 rows).
// fwd: stored forward PML displacements of the stage, per source
// [x1 u (3) | x2 u (3) | x0 u (3)] x sp on the PML shell.
template <typename R, int TX, int TY, int TZ>
__global__ void __launch_bounds__(PMLFWI_ETHREADS)
pml_gradient_kernel(Geo g, const Tile* __restrict__ tiles, int ntiles, int nsrc, const R* __restrict__ Ybase,
                    long long ystride, const R* __restrict__ fwd, long long fstride, double gw,
                    double* __restrict__ gacc, Part PG) {
  constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
  constexpr int NB = BX * BY * BZ, NP = 27 * TX * TY * TZ;
  static_assert(NB <= PMLFWI_ETHREADS, "one box node per thread");
  __shared__ R sW[9][NB];
  __shared__ R sZ[6][NB];
  __shared__ R sG[2][NP];
  __shared__ double sGacc[2][NB];

  const int ti = xcd_tile();
  if (ti >= ntiles) return;
  const Tile t = tiles[ti];
  const int cx = t.c & 255, cy = (t.c >> 8) & 255, cz = (t.c >> 16) & 255;
  const size_t np = (size_t)g.sp, nn = (size_t)g.sn;
  const R s2h = R(2.0 / g.h);

  const int n = threadIdx.x;
  const int lx = n % BX, ly = (n / BX) % BY, lz = n / (BX * BY);
  const bool live = n < NB && lx <= 2 * cx && ly <= 2 * cy && lz <= 2 * cz;
  const int gi = 2 * t.x + lx, gj = 2 * t.y + ly, gk = 2 * t.z + lz;
  R Le[3] = {0, 0, 0}, Lp[3] = {0, 0, 0}, Lw[3] = {0, 0, 0};
  bool hist = false, free_u = false;
  size_t gnode = 0, gp = 0;
  if (live) {
    pml_node_setup<R>(g, gi, gj, gk, Le, Lp, Lw, hist, gnode, gp);
    free_u = !is_dirichlet(g, gi, gj, gk);
    sGacc[0][n] = 0.0;
    sGacc[1][n] = 0.0;
  }
  for (int src = 0; src < nsrc; ++src) {
    if (live) {
      const R* F = fwd + (size_t)src * fstride;
      const R* P = Ybase + (size_t)src * ystride + 6 * nn;
      PmlNode<R> v;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        v.u1[d] = free_u ? F[d * np + gp] : R(0);
        v.u2[d] = free_u ? F[(3 + d) * np + gp] : R(0);
        v.u0[d] = (free_u && hist) ? F[(6 + d) * np + gp] : R(0);
      }
      pml_node_w<R, NB>(v, Le, Lp, Lw, n, sW);
#pragma unroll
      for (int c = 0; c < 6; ++c) sZ[c][n] = P[p_at(np, P_X1S + c, gp)];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NP; q += blockDim.x) {
      const int pt = q % 27, e = q / 27;
      const int ea = e % TX, eb = (e / TX) % TY, ec = e / (TX * TY);
      if (ea >= cx || eb >= cy || ec >= cz) continue;
      const int qa = pt % 3, qb = (pt / 3) % 3, qc = pt / 9;
      const int px = 2 * ea + qa, py = 2 * eb + qb, pz = 2 * ec + qc;
      const int nq = px + BX * (py + BY * pz);
      R H[3][3];
      const R xa = R(qa - 1), xb = R(qb - 1), xc = R(qc - 1);
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        R hx = 0, hy = 0, hz = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          hx += dbasis(xa, a) * sW[0 + ii][(2 * ea + a) + BX * (py + BY * pz)];
          hy += dbasis(xb, a) * sW[3 + ii][px + BX * ((2 * eb + a) + BY * pz)];
          hz += dbasis(xc, a) * sW[6 + ii][px + BX * (py + BY * (2 * ec + a))];
        }
        H[ii][0] = hx * s2h; H[ii][1] = hy * s2h; H[ii][2] = hz * s2h;
      }
      const R wq = R(0.125 * g.h * g.h * g.h * wlgl(qa) * wlgl(qb) * wlgl(qc));
      const R z0 = sZ[0][nq], z1 = sZ[1][nq], z2 = sZ[2][nq], z3 = sZ[3][nq], z4 = sZ[4][nq], z5 = sZ[5][nq];
      const R tr = H[0][0] + H[1][1] + H[2][2];
      R em = 2 * (z0 * H[0][0] + z1 * H[1][1] + z2 * H[2][2]);
      em += z3 * (H[1][2] + H[2][1]) + z4 * (H[0][2] + H[2][0]) + z5 * (H[0][1] + H[1][0]);
      sG[0][q] = -wq * tr * (z0 + z1 + z2);
      sG[1][q] = -wq * em;
    }
    __syncthreads();
    if (live) {
      int ox[2], oy[2], oz[2];
      bool vx[2], vy[2], vz[2];
      axis_bricks(lx, cx, 27, 1, ox, vx);
      axis_bricks(ly, cy, 27 * TX, 3, oy, vy);
      axis_bricks(lz, cz, 27 * TX * TY, 9, oz, vz);
      R gl = 0, gm = 0;
#pragma unroll
      for (int a3 = 0; a3 < 2; ++a3)
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int a1 = 0; a1 < 2; ++a1) {
            if (!(vx[a1] && vy[a2] && vz[a3])) continue;
            const int qn = ox[a1] + oy[a2] + oz[a3];
            gl += sG[0][qn];
            gm += sG[1][qn];
          }
      sGacc[0][n] += (double)gl;
      sGacc[1][n] += (double)gm;
    }
    __syncthreads();
  }
  if (live) {
    const int cs = (lx == 2 * cx) | ((ly == 2 * cy) << 1) | ((lz == 2 * cz) << 2);
    const size_t o = (size_t)PG.off[cs] + part_node(g, PG, cs, gi, gj, gk), gs = (size_t)PG.size[cs];
    const double a0 = gacc[o], a1 = gacc[o + gs];
    gacc[o] = a0 + gw * sGacc[0][n];
    gacc[o + gs] = a1 + gw * sGacc[1][n];
  }
}

// Nodal part of one RK4 stage.  With r the element residual of the stage input
// Y, the rates are K = (x1|PML, x2, M^{-1}(f - r - nodal PML terms)) and
//   mode 0:  acc = Xn + cA K,  Yout = Xn + cY K   (the stage input is Xn)
//   mode 1:  acc += cA K,      Yout = Xn + cY K
//   mode 2:  Xn = acc + cA K
template <typename R>
struct NodalArgs {
  const R* Yin;
  R* Yout;
  R* Xn;
  R* acc;
  const R* res;               // partial arrays of source 0
  Part part;
  const R* invMu;
  long long reg;
  R cA, cY;
  int mode;
  const int* src_node;        // nullptr: no load
  const double* src_dir;      // (nsrc, 3)
  const double* wav;          // (nsrc, wav_len)
  int wav_len, wav_idx;
  R* store;                   // x1 displacement ([si][3]) of the produced register on the
  long long store_stride;     // interior closure (per source stride), or nullptr
  R* pstore;                  // PML displacement fields of the produced register
  long long pstore_stride;    // [x1 u | x2 u | x0 u] x sp per source, or nullptr
  long long first, last;      // row range of this launch: [0, sn) node rows, then PML rows
  unsigned rot;               // workgroup b takes rows of block (b + rot) mod grid
};

// Where a node's contributions sit in the partial arrays: array 0 always, and
// array c != 0 when every axis of c is an upper-face axis of the node.
struct PartSlots {
  int mask;
  size_t nc[8];   // node index inside array c (c != 0: compressed box)
};

__device__ __forceinline__ PartSlots part_slots(const Geo& g, const Part& P, int i, int j, int k) {
  PartSlots S;
  const int fx = g.fo[i], fy = g.fo[ax_y(g) + j], fz = g.fo[ax_z(g) + k];
  S.mask = (fx >= 0) | ((fy >= 0) << 1) | ((fz >= 0) << 2);
#pragma unroll
  for (int c = 1; c < 8; ++c) {
    const int ii = (c & 1) ? fx : i, jj = (c & 2) ? fy : j, kk = (c & 4) ? fz : k;
    S.nc[c] = (size_t)ii + (size_t)P.nx[c] * ((size_t)jj + (size_t)P.ny[c] * kk);
  }
  return S;
}

// Sum over the partial arrays of a node's NR = 3 u-rows (SROWS false; base0 =
// 3 node) or NR = 6 S-rows (SROWS true; base0 = 3 sn + 6 p), each array's rows
// read as one contiguous vector.  The single-axis arrays (c = 1, 2, 4) are read
// unconditionally, at their first node when the node is not on that face, and
// the values are discarded by a select: the loads then issue together with the
// others instead of one branch at a time.  Nodes on two or three faces (1/32
// of the nodes or fewer per array) take a branch.
template <typename R, int NR, bool SROWS>
__device__ __forceinline__ void gather_rows(const Part& P, const PartSlots& S, const R* res, size_t base0,
                                            R out[NR]) {
  auto first = [&](int c, size_t n) {
    return (size_t)P.off[c] + (SROWS ? 3 * (size_t)P.size[c] + 6 * n : 3 * n);
  };
  R t[3][NR];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int c = 1 << b;
    const bool on = (S.mask & c) != 0;
    const size_t o = first(c, on ? S.nc[c] : 0);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const R v = res[o + r];
      t[b][r] = on ? v : R(0);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) out[r] = __builtin_nontemporal_load(&res[base0 + r]) + t[0][r] + t[1][r] + t[2][r];
  if (S.mask == 3 || S.mask == 5 || S.mask == 6 || S.mask == 7) {
#pragma unroll
    for (int c = 3; c < 8; ++c)
      if (c != 4 && (S.mask & c) == c) {
        const size_t o = first(c, S.nc[c]);
#pragma unroll
        for (int r = 0; r < NR; ++r) out[r] += res[o + r];
      }
  }
}

// Nodal part of one stage for node rows and PML rows; MODE as described above,
// STORE >= 1 writes the produced x1 displacement on the interior closure,
// STORE = 2 also the PML displacement fields (full gradient).
// Threads [0, sn) take the displacement rows of node gid (none past n_nodes),
// threads [sn, sn + n_pml) the PML rows; every load of a thread is issued
// before its first store.  The accumulator and the kept stage displacement
// are written, and Xn, the stage input and the residual partials are read,
// with non-temporal hints: none of them is touched again before the next
// stage's nodal pass (the kept displacement not before the adjoint), so they
// should not displace the stage output that the next element launches read.
template <typename R, int MODE, int STORE>
__global__ void __launch_bounds__(PMLFWI_NODAL_THREADS) nodal_rk_kernel(Geo g, NodalArgs<R> A) {
  const int src = blockIdx.y;
  const unsigned blk = A.rot ? (blockIdx.x + A.rot) % gridDim.x : blockIdx.x;
  const long long gid = A.first + (long long)blk * blockDim.x + threadIdx.x;
  if (gid >= A.last) return;
  const size_t nn = (size_t)g.sn, np = (size_t)g.sp;
  const R* __restrict__ Y = A.Yin + (size_t)src * A.reg;
  R* __restrict__ Yo = MODE == 2 ? nullptr : A.Yout + (size_t)src * A.reg;
  R* __restrict__ X = A.Xn + (size_t)src * A.reg;
  R* __restrict__ C = A.acc + (size_t)src * A.reg;
  const R* __restrict__ res = A.res + (size_t)src * A.part.per_src;
  const R cA = A.cA, cY = A.cY;

  if (gid < (long long)nn) {
    if (gid >= g.n_nodes) return;
    const int node = (int)gid;
    const int k = node / g.plane;
    const int r_ = node - k * g.plane;
    const int j = r_ / g.NX, i = r_ - j * g.NX;
    if (is_dirichlet(g, i, j, k)) return;
    const bool pml = in_pml(g, i, j, k);
    const PartSlots PS = part_slots(g, A.part, i, j, k);
    R u1[3], u2[3], rr[3], x1[3], x2[3], c1[3], c2[3];
    gather_rows<R, 3, false>(A.part, PS, res, 3 * (size_t)node, rr);
    const size_t o1 = u_at(nn, 0, node), o2 = u_at(nn, 3, node);   // x1 u, x2 u of the node
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u1[d] = __builtin_nontemporal_load(&Y[o1 + d]);
      u2[d] = __builtin_nontemporal_load(&Y[o2 + d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (MODE == 1) x1[d] = __builtin_nontemporal_load(&X[o1 + d]);
      if (MODE == 0) x1[d] = u1[d];   // the first stage's input is Xn itself
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (MODE == 1) x2[d] = __builtin_nontemporal_load(&X[o2 + d]);
      if (MODE == 0) x2[d] = u2[d];
    }
    if (MODE != 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) c1[d] = C[o1 + d];
#pragma unroll
      for (int d = 0; d < 3; ++d) c2[d] = C[o2 + d];
    }
    const R im = A.invMu[node];
    R a2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) a2[d] = -im * rr[d];
    if (A.src_node && A.src_node[src] == node) {
      const double s = A.wav[(size_t)src * A.wav_len + A.wav_idx];
#pragma unroll
      for (int d = 0; d < 3; ++d) a2[d] += im * R(A.src_dir[3 * src + d] * s);
    }
    if (pml) {
      double mrd, mp;
      lumped_masses_tab(g, i, j, k, mrd, mp);
      const PmlCoef c = pml_coef_tab(g, i, j, k);
      const R kap = R(mp) / (R(mrd) + R(c.a) * R(mp));
      R u0[3] = {0, 0, 0};
      if (c.nbeta >= 2) {
        const size_t p = (size_t)pml_index(g, i, j, k);
        const R* P = Y + 6 * nn + p_at(np, P_X0U, p);
#pragma unroll
        for (int d = 0; d < 3; ++d) u0[d] = P[d];
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
        a2[d] -= kap * (R(c.b) * u2[d] + R(c.c) * u1[d] + R(c.d) * u0[d]);
    }
    // each field's three components are stored together (one vector store)
    R out1[3], out2[3], n1[3], n2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (MODE == 2) {
        out1[d] = c1[d] + cA * u2[d];
        out2[d] = c2[d] + cA * a2[d];
      } else {
        n1[d] = (MODE == 0 ? x1[d] : c1[d]) + cA * u2[d];
        n2[d] = (MODE == 0 ? x2[d] : c2[d]) + cA * a2[d];
        out1[d] = x1[d] + cY * u2[d];
        out2[d] = x2[d] + cY * a2[d];
      }
    }
    R* const D = MODE == 2 ? X : Yo;
#pragma unroll
    for (int d = 0; d < 3; ++d) D[o1 + d] = out1[d];
#pragma unroll
    for (int d = 0; d < 3; ++d) D[o2 + d] = out2[d];
    if (MODE != 2) {
#pragma unroll
      for (int d = 0; d < 3; ++d) __builtin_nontemporal_store(n1[d], &C[o1 + d]);
#pragma unroll
      for (int d = 0; d < 3; ++d) __builtin_nontemporal_store(n2[d], &C[o2 + d]);
    }
    if (STORE == 2 && pml) {
      R* PS_ = A.pstore + (size_t)src * A.pstore_stride;
      const size_t p = (size_t)pml_index(g, i, j, k);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        PS_[(size_t)d * np + p] = out1[d];
        PS_[(size_t)(3 + d) * np + p] = out2[d];
      }
    }
    if (STORE) {
      const int mi = interior_index(g, i, j, k);
      if (mi >= 0) {
        R* S = A.store + (size_t)src * A.store_stride;
#pragma unroll
        for (int d = 0; d < 3; ++d) __builtin_nontemporal_store(out1[d], &S[3 * (size_t)mi + d]);
      }
    }
    return;
  }
  const long long pp = gid - (long long)nn;
  if (pp >= (long long)g.n_pml) return;
  const size_t p = (size_t)pp;
  int i, j, k;
  pml_coords(g, (int)p, i, j, k);
  const PmlCoef c = pml_coef_tab(g, i, j, k);
  double mrd, mp;
  lumped_masses_tab(g, i, j, k, mrd, mp);
  const bool hist = c.nbeta >= 2;
  const bool hu = hist && !is_dirichlet(g, i, j, k);
  const R* PY = Y + 6 * nn;
  R* PX = X + 6 * nn;
  R* PC = C + 6 * nn;
  R* PO = MODE == 2 ? nullptr : Yo + 6 * nn;
  const PartSlots PS = part_slots(g, A.part, i, j, k);
  const R ia = R(1) / R(c.a), iam = R(1) / (R(c.a) * R(mp));
  const R cb = R(c.b), cc = R(c.c), cd = R(c.d);

  // Rates of the PML components, then the register updates, one field at a
  // time (x0 u: 3 components, on history nodes off the Dirichlet boundary;
  // x0 S: 6, on history nodes; x1 S, x2 S: 6 each), so that a field's
  // components move with one vector load or store.
  const size_t b0u = p_at(np, P_X0U, p), b0s = p_at(np, P_X0S, p);
  const size_t b1s = p_at(np, P_X1S, p), b2s = p_at(np, P_X2S, p);
  R s0[6], s1[6], s2[6], rv[6], y1[3];
#pragma unroll
  for (int v = 0; v < 6; ++v) s1[v] = __builtin_nontemporal_load(&PY[b1s + v]);
#pragma unroll
  for (int v = 0; v < 6; ++v) s2[v] = __builtin_nontemporal_load(&PY[b2s + v]);
  if (hist) {
#pragma unroll
    for (int v = 0; v < 6; ++v) s0[v] = __builtin_nontemporal_load(&PY[b0s + v]);
  } else {
#pragma unroll
    for (int v = 0; v < 6; ++v) s0[v] = R(0);
  }
  gather_rows<R, 6, true>(A.part, PS, res, 3 * nn + 6 * p, rv);
  if (hu) {
    const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
#pragma unroll
    for (int d = 0; d < 3; ++d) y1[d] = Y[u_at(nn, 0, node) + d];
  }
  // register values of one field: Xn (mode 0: the stage input) and acc
  auto fetch = [&](size_t b, const R* in, auto& xv, auto& cv) {
    constexpr int n = sizeof(xv) / sizeof(R);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (MODE == 0) xv[q] = in ? in[q] : __builtin_nontemporal_load(&PX[b + q]);
      if (MODE == 1) xv[q] = __builtin_nontemporal_load(&PX[b + q]);
    }
    if (MODE != 0) {
#pragma unroll
      for (int q = 0; q < n; ++q) cv[q] = PC[b + q];
    }
  };
  // stage combination of one field with its rates; out: the produced value
  auto update = [&](size_t b, const auto& xv, const auto& cv, const auto& rate, auto& out) {
    constexpr int n = sizeof(xv) / sizeof(R);
    R na[n];
#pragma unroll
    for (int q = 0; q < n; ++q) {
      if (MODE == 2) {
        out[q] = cv[q] + cA * rate[q];
      } else {
        na[q] = (MODE == 0 ? xv[q] : cv[q]) + cA * rate[q];
        out[q] = xv[q] + cY * rate[q];
      }
    }
    R* const D = MODE == 2 ? PX : PO;
#pragma unroll
    for (int q = 0; q < n; ++q) D[b + q] = out[q];
    if (MODE != 2) {
#pragma unroll
      for (int q = 0; q < n; ++q) __builtin_nontemporal_store(na[q], &PC[b + q]);
    }
  };
  R x0u[3], c0u[3], x0s[6], c0s[6], x1s[6], c1s[6], x2s[6], c2s[6];
  if (hu) fetch(b0u, nullptr, x0u, c0u);
  if (hist) fetch(b0s, s0, x0s, c0s);
  fetch(b1s, s1, x1s, c1s);
  fetch(b2s, s2, x2s, c2s);
  R r2s[6], o6[6], o3[3];
#pragma unroll
  for (int v = 0; v < 6; ++v) r2s[v] = -rv[v] * iam - ia * (cb * s2[v] + cc * s1[v] + cd * s0[v]);
  if (hu) {
    update(b0u, x0u, c0u, y1, o3);
    if (STORE == 2) {   // x0 u of a history node
#pragma unroll
      for (int d = 0; d < 3; ++d) A.pstore[(size_t)src * A.pstore_stride + (size_t)(6 + d) * np + p] = o3[d];
    }
  }
  if (hist) update(b0s, x0s, c0s, s1, o6);
  update(b1s, x1s, c1s, s2, o6);
  update(b2s, x2s, c2s, r2s, o6);
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
  lumped_masses_tab(g, i, j, k, mrd, mp);
  const PmlCoef c = pml_coef_tab(g, i, j, k);
  invMu[node] = R(1.0 / (rho[material_index(g, i, j, k)] * (mrd + c.a * mp)));
}

}  // namespace pmlfwi
