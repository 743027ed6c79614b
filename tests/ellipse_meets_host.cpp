// Host driver for the CPU test of the render kernels' culling test
// (ellipse_meets / tile_kept in csrc/common.hpp, compiled for the host):
// reads cases from stdin, writes one 0/1 answer per case to stdout.
// Case: u_hi v_hi u_lo v_lo A B C lo x0 x1 y0 y1 log2_alpha
#include <cstdio>

#include "../paper_2411_12788_amd/csrc/common.hpp"

int main() {
  float u, v, ul, vl, A, B, C, lo, la;
  int x0, x1, y0, y1;
  while (std::scanf("%a %a %a %a %a %a %a %a %d %d %d %d %a", &u, &v, &ul, &vl, &A, &B, &C, &lo, &x0, &x1, &y0, &y1,
                    &la) == 13) {
    const float4 r0 = make_float4(u, v, ul, vl), r1 = make_float4(A, B, C, lo);
    std::printf("%d\n", msplat::ellipse_meets(r0, r1, x0, x1, y0, y1, la) ? 1 : 0);
  }
  return 0;
}
