// Structured-grid geometry, node classes and PML coefficients (device side).
//
// Mesh (Fig. 3 of arXiv:1504.08340): interior box [-Lx/2,Lx/2]x[-Ly/2,Ly/2]x
// [-Lz,0] of ex*ey*ez cubic 27-node bricks of edge h, a PML of ps bricks on
// +-x, +-y and pb bricks below; u = 0 on the outer sides and bottom (2c).
//
// Index spaces
//   full grid   : node id = i + NX*(j + NY*k), k = 0 at the PML bottom.
//   PML shell   : every node of a PML brick (the closed PML), numbered plane by
//                 plane: planes k <= zb = 2*pb are complete; above them only the
//                 frame of width w = 2*ps+1 nodes (full rows j < w and
//                 j >= NY-w, the two end blocks of the rows in between).
//   interior    : the closed interior box (material grid), id jx+NIX*(jy+NIY*jz).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmlfwi {

struct Geo {
  int NX, NY, NZ;        // full node grid
  int EX, EY, EZ;        // bricks
  int ex, ey, ez;        // interior bricks
  int ps, pb;            // PML bricks on the sides / at the bottom
  int NIX, NIY, NIZ;     // interior-closure node grid
  int w, zb;             // frame width (nodes), last complete PML plane
  int n_nodes, n_pml, n_int;
  int sn, sp, si;        // component strides of the three index spaces: the
                         // counts rounded up to 64 entries, so that every
                         // component array starts on a 256-byte boundary
  int plane, ring;       // NX*NY, nodes of one frame plane
  double h;
  double x0, y0, z0;     // coordinates of node (0,0,0)
  double hx, hy, hz;     // interior half widths (x,y) and depth (z)
  double Lps, Lpb;       // PML thickness on the sides / at the bottom
  double alpha0, beta0;
  int m;
  // device tables, [NX + NY + NZ] entries per quantity, axes x | y | z:
  //   tab: alpha, beta (PML profile), total and interior 1D lumped-mass factors
  //   fo : ordinal of an index among the upper faces of the tile lattice, or -1
  const double* tab;
  const int* fo;
};

// Per-axis offsets into the [NX + NY + NZ] tables.
__host__ __device__ inline int ax_y(const Geo& g) { return g.NX; }
__host__ __device__ inline int ax_z(const Geo& g) { return g.NX + g.NY; }
__host__ __device__ inline int ax_n(const Geo& g) { return g.NX + g.NY + g.NZ; }

__host__ __device__ inline bool is_dirichlet(const Geo& g, int i, int j, int k) {
  return i == 0 || i == g.NX - 1 || j == 0 || j == g.NY - 1 || k == 0;
}

__host__ __device__ inline bool in_pml(const Geo& g, int i, int j, int k) {
  return k <= g.zb || j < g.w || j >= g.NY - g.w || i < g.w || i >= g.NX - g.w;
}

__host__ __device__ inline int pml_index(const Geo& g, int i, int j, int k) {
  if (k <= g.zb) return k * g.plane + j * g.NX + i;
  const int base = (g.zb + 1) * g.plane + (k - g.zb - 1) * g.ring;
  const int w = g.w;
  if (j < w) return base + j * g.NX + i;
  if (j >= g.NY - w)
    return base + w * g.NX + (g.NY - 2 * w) * 2 * w + (j - (g.NY - w)) * g.NX + i;
  return base + w * g.NX + (j - w) * 2 * w + (i < w ? i : i - (g.NX - 2 * w));
}

__host__ __device__ inline void pml_coords(const Geo& g, int p, int& i, int& j, int& k) {
  const int nfull = (g.zb + 1) * g.plane;
  if (p < nfull) {
    k = p / g.plane;
    const int r = p - k * g.plane;
    j = r / g.NX;
    i = r - j * g.NX;
    return;
  }
  const int q = p - nfull;
  const int kk = q / g.ring;
  k = g.zb + 1 + kk;
  int r = q - kk * g.ring;
  const int w = g.w;
  if (r < w * g.NX) {
    j = r / g.NX;
    i = r - j * g.NX;
    return;
  }
  r -= w * g.NX;
  if (r < (g.NY - 2 * w) * 2 * w) {
    const int jj = r / (2 * w);
    j = w + jj;
    const int c = r - jj * 2 * w;
    i = c < w ? c : g.NX - 2 * w + c;
    return;
  }
  r -= (g.NY - 2 * w) * 2 * w;
  j = g.NY - w + r / g.NX;
  i = r - (r / g.NX) * g.NX;
}

// Material of a node: interior-closure value at its projection onto the box
// (the interface value carried into the PML).
__host__ __device__ inline int material_index(const Geo& g, int i, int j, int k) {
  int jx = i - 2 * g.ps, jy = j - 2 * g.ps, jz = k - 2 * g.pb;
  jx = jx < 0 ? 0 : (jx >= g.NIX ? g.NIX - 1 : jx);
  jy = jy < 0 ? 0 : (jy >= g.NIY ? g.NIY - 1 : jy);
  jz = jz < 0 ? 0 : (jz >= g.NIZ ? g.NIZ - 1 : jz);
  return jx + g.NIX * (jy + g.NIY * jz);
}

// Interior-closure id of a node inside the closed box, or -1.
__host__ __device__ inline int interior_index(const Geo& g, int i, int j, int k) {
  const int jx = i - 2 * g.ps, jy = j - 2 * g.ps, jz = k - 2 * g.pb;
  if (jx < 0 || jx >= g.NIX || jy < 0 || jy >= g.NIY || jz < 0 || jz >= g.NIZ) return -1;
  return jx + g.NIX * (jy + g.NIY * jz);
}

// PML profile along one axis: xi = distance into the layer.
__host__ __device__ inline void stretch(const Geo& g, double xi, double L, double& a, double& b) {
  if (xi <= 0.0 || L <= 0.0) {
    a = 1.0;
    b = 0.0;
    return;
  }
  const double r = xi / L;
  double rm = 1.0;
  for (int t = 0; t < g.m; ++t) rm *= r;
  a = 1.0 + g.alpha0 * rm;
  b = g.beta0 * rm;
}

// Stretch tensors Lambda_e, Lambda_p, Lambda_w (diagonals) and scalars
// a, b, c, d at a node, from eps_s = alpha_s + beta_s/(i w):
//   Lambda(w) = diag(eps_x eps_y eps_z / eps_k),  eps_x eps_y eps_z = a + b/(iw) + ...
struct PmlCoef {
  double Le[3], Lp[3], Lw[3];
  double a, b, c, d;
  int nbeta;               // number of axes with beta > 0 (history is used iff >= 2)
};

__host__ __device__ inline PmlCoef pml_coef(const Geo& g, int i, int j, int k) {
  const double x = g.x0 + 0.5 * g.h * i, y = g.y0 + 0.5 * g.h * j, z = g.z0 + 0.5 * g.h * k;
  double ax, bx, ay, by, az, bz;
  stretch(g, fabs(x) - g.hx, g.Lps, ax, bx);
  stretch(g, fabs(y) - g.hy, g.Lps, ay, by);
  stretch(g, -z - g.hz, g.Lpb, az, bz);
  PmlCoef c;
  c.Le[0] = ay * az; c.Lp[0] = ay * bz + by * az; c.Lw[0] = by * bz;
  c.Le[1] = ax * az; c.Lp[1] = ax * bz + bx * az; c.Lw[1] = bx * bz;
  c.Le[2] = ax * ay; c.Lp[2] = ax * by + bx * ay; c.Lw[2] = bx * by;
  c.a = ax * ay * az;
  c.b = ax * ay * bz + ax * by * az + bx * ay * az;
  c.c = ax * by * bz + bx * ay * bz + bx * by * az;
  c.d = bx * by * bz;
  c.nbeta = (bx > 0.0) + (by > 0.0) + (bz > 0.0);
  return c;
}

// Same coefficients from the per-axis tables (no division or power on device).
__device__ __forceinline__ PmlCoef pml_coef_tab(const Geo& g, int i, int j, int k) {
  const int nt = ax_n(g);
  const double* A = g.tab;
  const double* B = g.tab + nt;
  const double ax = A[i], ay = A[ax_y(g) + j], az = A[ax_z(g) + k];
  const double bx = B[i], by = B[ax_y(g) + j], bz = B[ax_z(g) + k];
  PmlCoef c;
  c.Le[0] = ay * az; c.Lp[0] = ay * bz + by * az; c.Lw[0] = by * bz;
  c.Le[1] = ax * az; c.Lp[1] = ax * bz + bx * az; c.Lw[1] = bx * bz;
  c.Le[2] = ax * ay; c.Lp[2] = ax * by + bx * ay; c.Lw[2] = bx * by;
  c.a = ax * ay * az;
  c.b = ax * ay * bz + ax * by * az + bx * ay * az;
  c.c = ax * by * bz + bx * ay * bz + bx * by * az;
  c.d = bx * by * bz;
  c.nbeta = (bx > 0.0) + (by > 0.0) + (bz > 0.0);
  return c;
}

// One-dimensional lumped-mass factors: sum of LGL weights of the bricks of
// [elo, ehi) that contain node l (weights 1/3, 4/3, 1/3).
__host__ __device__ inline double mass1d(int l, int elo, int ehi) {
  double s = 0.0;
  if (l & 1) {
    const int e = (l - 1) >> 1;
    if (e >= elo && e < ehi) s += 4.0 / 3.0;
  } else {
    const int e1 = (l >> 1) - 1, e2 = l >> 1;
    if (e1 >= elo && e1 < ehi) s += 1.0 / 3.0;
    if (e2 >= elo && e2 < ehi) s += 1.0 / 3.0;
  }
  return s;
}

// Lumped masses of a node: m_rd over interior bricks, m_p over PML bricks.
__host__ __device__ inline void lumped_masses(const Geo& g, int i, int j, int k, double& mrd, double& mp) {
  const double v = 0.125 * g.h * g.h * g.h;
  const double tot = v * mass1d(i, 0, g.EX) * mass1d(j, 0, g.EY) * mass1d(k, 0, g.EZ);
  mrd = v * mass1d(i, g.ps, g.ps + g.ex) * mass1d(j, g.ps, g.ps + g.ey) * mass1d(k, g.pb, g.EZ);
  mp = tot - mrd;
}

__device__ __forceinline__ void lumped_masses_tab(const Geo& g, int i, int j, int k, double& mrd, double& mp) {
  const int nt = ax_n(g);
  const double* T = g.tab + 2 * nt;
  const double* D = g.tab + 3 * nt;
  const double v = 0.125 * g.h * g.h * g.h;
  const double tot = v * T[i] * T[ax_y(g) + j] * T[ax_z(g) + k];
  mrd = v * D[i] * D[ax_y(g) + j] * D[ax_z(g) + k];
  mp = tot - mrd;
}

}  // namespace pmlfwi
