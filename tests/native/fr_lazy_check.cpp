// Host check of the lazy-reduction field routines: reads lines of
// "k a_1 b_1 ... a_k b_k" (decimal-free: 64 hex digits per operand, Montgomery
// limbs as stored) and prints, per line, the reduced Montgomery value of
// sum_i a_i b_i R^{-1} as 64 hex digits, and the plain product sum for k = 2
// through fr_mul_add2 on a second line.
#include <cstdio>
#include <cstring>
#include <string>

#include "../../paper_2404_10404_amd/csrc/fr.hpp"

using namespace gkr;

static Fr parse(const char* h) {
  Fr r;
  for (int k = 0; k < 8; ++k) {
    char buf[9];
    memcpy(buf, h + (7 - k) * 8, 8);
    buf[8] = 0;
    r.v[k] = (uint32_t)strtoul(buf, nullptr, 16);
  }
  return r;
}

static void print(const Fr& a) {
  for (int k = 7; k >= 0; --k) printf("%08x", a.v[k]);
  printf("\n");
}

template <int T>
static Fr reduce_n(const FrWide& A) { return frw_reduce<T>(A); }

static Fr reduce_dyn(const FrWide& A, int k) {
  switch (k) {
#define C(n) case n: return reduce_n<n>(A);
    C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)
#undef C
  }
  return fr_zero();
}

int main() {
  int k;
  char a[80], b[80];
  while (scanf("%d", &k) == 1) {
    FrWide A = frw_zero();
    FrCols C = frc_zero();
    Fr first[2][2];
    for (int i = 0; i < k; ++i) {
      if (scanf("%64s %64s", a, b) != 2) return 1;
      Fr x = parse(a), y = parse(b);
      if (i < 2) { first[i][0] = x; first[i][1] = y; }
      frw_mac(A, x, y);
      frc_mac(C, x, y);
    }
    print(reduce_dyn(A, k));
    print(reduce_dyn(frc_wide(C), k));
    if (k == 2) print(fr_mul_add2(first[0][0], first[0][1], first[1][0], first[1][1]));
    if (k == 1) print(fr_half(first[0][1]));
  }
  return 0;
}
