/*
 * Bulk field operations for the CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Plain C, independent of the HIP library: elements are canonical values
 * in [0, p) as four little-endian 64-bit words. A product is formed by
 * schoolbook multiplication into eight words and reduced by replacing each
 * word w_k at position k >= 4 with w_k * (2^(64k) mod p), repeating until the
 * value fits in 256 bits, then subtracting p while the value is >= p. The
 * residues 2^(64k) mod p are computed at start-up by repeated doubling.
 *
 * The folds of one round are independent and run on OpenMP threads.
 *
 * Used for the multilinear extension of large input vectors (GKR section:
 * V~(r) = sum_b V[b] eq(r, b), evaluated by binding variable 1 first) where
 * the pure-Python oracle would take minutes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static const uint64_t P[4] = {0x43e1f593f0000001ULL, 0x2833e84879b97091ULL, 0xb85045b68181585dULL,
                              0x30644e72e131a029ULL};
static uint64_t RES[8][4]; /* RES[k] = 2^(64k) mod p, k = 0..7 */
static int ready = 0;

static int geq_p(const uint64_t a[4]) {
  for (int k = 3; k >= 0; --k) {
    if (a[k] > P[k]) return 1;
    if (a[k] < P[k]) return 0;
  }
  return 1;
}

static void sub_p(uint64_t a[4]) {
  uint64_t br = 0;
  for (int k = 0; k < 4; ++k) {
    u128 d = (u128)a[k] - P[k] - br;
    a[k] = (uint64_t)d;
    br = (uint64_t)(d >> 64) ? 1 : 0;
  }
}

/* a = 2a mod p for a < p */
static void dbl(uint64_t a[4]) {
  uint64_t top = a[3] >> 63;
  for (int k = 3; k > 0; --k) a[k] = (a[k] << 1) | (a[k - 1] >> 63);
  a[0] <<= 1;
  if (top || geq_p(a)) sub_p(a);
}

static void init(void) {
  if (ready) return;
  uint64_t x[4] = {1, 0, 0, 0};
  for (int k = 0; k < 8; ++k) {
    memcpy(RES[k], x, sizeof(x));
    for (int b = 0; b < 64; ++b) dbl(x);
  }
  ready = 1;
}

/* Reduce a value given as `n` 64-bit words (n <= 8) modulo p. */
static void reduce(const uint64_t* w, int n, uint64_t out[4]) {
  uint64_t acc[6];
  uint64_t cur[8];
  int len = n;
  memcpy(cur, w, (size_t)n * 8);
  while (len > 4) {
    memset(acc, 0, sizeof(acc));
    for (int k = 0; k < 4; ++k) { /* low words as they are */
      u128 s = (u128)acc[k] + cur[k];
      acc[k] = (uint64_t)s;
      uint64_t c = (uint64_t)(s >> 64);
      for (int j = k + 1; c && j < 6; ++j) {
        s = (u128)acc[j] + c;
        acc[j] = (uint64_t)s;
        c = (uint64_t)(s >> 64);
      }
    }
    for (int k = 4; k < len; ++k) { /* high word k contributes cur[k] * RES[k] */
      uint64_t carry = 0;
      for (int j = 0; j < 4; ++j) {
        u128 s = (u128)cur[k] * RES[k][j] + acc[j] + carry;
        acc[j] = (uint64_t)s;
        carry = (uint64_t)(s >> 64);
      }
      for (int j = 4; carry && j < 6; ++j) {
        u128 s = (u128)acc[j] + carry;
        acc[j] = (uint64_t)s;
        carry = (uint64_t)(s >> 64);
      }
    }
    len = 6;
    while (len > 4 && acc[len - 1] == 0) --len;
    memcpy(cur, acc, sizeof(acc));
  }
  for (int k = len; k < 4; ++k) cur[k] = 0;
  memcpy(out, cur, 32);
  while (geq_p(out)) sub_p(out);
}

static void mulmod(const uint64_t a[4], const uint64_t b[4], uint64_t out[4]) {
  uint64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 4; ++i) {
    uint64_t carry = 0;
    for (int j = 0; j < 4; ++j) {
      u128 s = (u128)a[i] * b[j] + t[i + j] + carry;
      t[i + j] = (uint64_t)s;
      carry = (uint64_t)(s >> 64);
    }
    t[i + 4] = carry;
  }
  reduce(t, 8, out);
}

static void addmod(const uint64_t a[4], const uint64_t b[4], uint64_t out[4]) {
  uint64_t t[5];
  uint64_t c = 0;
  for (int k = 0; k < 4; ++k) {
    u128 s = (u128)a[k] + b[k] + c;
    t[k] = (uint64_t)s;
    c = (uint64_t)(s >> 64);
  }
  t[4] = c;
  reduce(t, 5, out);
}

static void submod(const uint64_t a[4], const uint64_t b[4], uint64_t out[4]) {
  /* a - b = a + (p - b) */
  uint64_t nb[4];
  uint64_t br = 0;
  for (int k = 0; k < 4; ++k) {
    u128 d = (u128)P[k] - b[k] - br;
    nb[k] = (uint64_t)d;
    br = (uint64_t)(d >> 64) ? 1 : 0;
  }
  addmod(a, nb, out);
}

/* out = a * b mod p for `count` pairs (used by the tests to pin this file). */
void oracle_mulmod_many(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t count) {
  init();
  for (uint64_t i = 0; i < count; ++i) mulmod(a + 4 * i, b + 4 * i, out + 4 * i);
}

void oracle_addsub_many(const uint64_t* a, const uint64_t* b, uint64_t* sum, uint64_t* diff,
                        uint64_t count) {
  init();
  for (uint64_t i = 0; i < count; ++i) {
    addmod(a + 4 * i, b + 4 * i, sum + 4 * i);
    submod(a + 4 * i, b + 4 * i, diff + 4 * i);
  }
}

/*
 * V~(r): `values` holds 2^k canonical elements, `r` k canonical elements
 * (variable 1 first). scratch must hold 2^(k-1) elements (k >= 1).
 * X'[b] = X[b] + r_j (X[b + M/2] - X[b]) for j = 1..k; the result is X[0].
 */
void oracle_mle(const uint64_t* values, uint32_t k, const uint64_t* r, uint64_t* scratch,
                uint64_t* out) {
  init();
  if (k == 0) {
    memcpy(out, values, 32);
    return;
  }
  uint64_t half = 1ULL << (k - 1);
  const uint64_t* src = values;
  for (uint32_t j = 0; j < k; ++j) {
#pragma omp parallel for schedule(static) if (half >= 4096)
    for (uint64_t b = 0; b < half; ++b) {
      uint64_t d[4], m[4];
      submod(src + 4 * (b + half), src + 4 * b, d);
      mulmod(r + 4 * j, d, m);
      addmod(src + 4 * b, m, scratch + 4 * b);
    }
    src = scratch;
    half >>= 1;
  }
  memcpy(out, scratch, 32);
}

/*
 * f(x) = sum_b c[b] x^b for `count` canonical coefficients c (the committed
 * polynomial of the input-layer commitment), x canonical: Horner's rule over
 * blocks of 2^16 coefficients, the block values combined by powers of x.
 */
void oracle_poly_eval(const uint64_t* coeffs, uint64_t count, const uint64_t* x, uint64_t* out) {
  init();
  const uint64_t B = 1ULL << 16;
  const uint64_t nblocks = (count + B - 1) / B;
  uint64_t* part = (uint64_t*)calloc(nblocks * 4 ? nblocks * 4 : 4, sizeof(uint64_t));
#pragma omp parallel for schedule(static) if (nblocks > 1)
  for (uint64_t blk = 0; blk < nblocks; ++blk) {
    uint64_t acc[4] = {0, 0, 0, 0}, t[4];
    const uint64_t lo = blk * B, hi = (lo + B < count) ? lo + B : count;
    for (uint64_t i = hi; i-- > lo;) {
      mulmod(acc, x, t);
      addmod(t, coeffs + 4 * i, acc);
    }
    memcpy(part + 4 * blk, acc, 32);
  }
  /* x^B, then sum_blk part[blk] (x^B)^blk by Horner over the blocks */
  uint64_t xb[4], t[4], acc[4] = {0, 0, 0, 0};
  memcpy(xb, x, 32);
  for (int k = 0; k < 16; ++k) {
    mulmod(xb, xb, t);
    memcpy(xb, t, 32);
  }
  for (uint64_t blk = nblocks; blk-- > 0;) {
    mulmod(acc, xb, t);
    addmod(t, part + 4 * blk, acc);
  }
  memcpy(out, acc, 32);
  free(part);
}
