// Host-side check of the state-register layout helpers (u_at, p_at): every
// (component, node) pair of a register maps to its own entry, the entries
// fill [0, 6 sn + 21 sp) exactly, and a field's components at one node are
// adjacent (so kernels move them as one vector).  Built for the host only.
#include "kernels.h"

#include <cstdio>
#include <vector>

static int check(size_t nn, size_t np) {
  using namespace pmlfwi;
  std::vector<int> hit(U_NCOMP * nn + P_NCOMP * np, 0);
  for (size_t n = 0; n < nn; ++n)
    for (int d = 0; d < U_NCOMP; ++d) hit[u_at(nn, d, n)]++;
  for (size_t p = 0; p < np; ++p)
    for (int q = 0; q < P_NCOMP; ++q) hit[U_NCOMP * nn + p_at(np, q, p)]++;
  for (size_t i = 0; i < hit.size(); ++i)
    if (hit[i] != 1) {
      std::printf("sn %zu sp %zu: entry %zu used %d times\n", nn, np, i, hit[i]);
      return 1;
    }
  const int first[5] = {0, 3, P_X0S, P_X1S, P_X2S};   // x2 u, then the PML fields
  for (size_t n = 0; n < nn; ++n) {
    for (int d = 1; d < 3; ++d)
      if (u_at(nn, d, n) != u_at(nn, 0, n) + d || u_at(nn, 3 + d, n) != u_at(nn, 3, n) + d) {
        std::printf("u components of node %zu not adjacent\n", n);
        return 1;
      }
  }
  for (size_t p = 0; p < np; ++p)
    for (int f = 2; f < 5; ++f)
      for (int v = 1; v < 6; ++v)
        if (p_at(np, first[f] + v, p) != p_at(np, first[f], p) + v) {
          std::printf("PML field %d of node %zu not adjacent\n", f, p);
          return 1;
        }
  return 0;
}

int main() {
  const size_t sizes[][2] = {{64, 64}, {128, 64}, {64 * 7, 64 * 3}, {520256, 270656}};
  for (const auto& s : sizes)
    if (check(s[0], s[1])) return 1;
  std::printf("layout ok\n");
  return 0;
}
