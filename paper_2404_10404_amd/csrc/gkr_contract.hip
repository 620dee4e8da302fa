// The phase-2 copy contraction on the matrix cores (Section 2.3, phase 2 of a
// data-parallel layer with the copy factors kept apart): for every
// sub-circuit wire y,
//   P[y] = sum_c U[c] W[y,c] R^-1 mod p,   Q[y] = sum_c V[c] W[y,c] R^-1 mod p
// (Montgomery forms), the same values the scalar contraction computes with
// lazy Montgomery products.
//
// The sums are exact integer sums of byte products. With W_j, U_i the bytes
// of W[y,c] and U[c] (little endian, 32 each),
//   sum_c U[c] W[y,c] = sum_k 2^(8k) E_k,  E_k = sum_c sum_{i + j = k} U_i[c] W_j[y,c],
// which is one matrix product: A[y][(c,j)] = W_j[y,c] is the table itself
// (row y is 32 * 2^n consecutive bytes), and B[(c,j)][k] = U_(k-j)[c] (zero
// outside 0 <= k - j < 32) is a banded matrix built from U. Columns 0..62 of
// B hold the bands of U, 64..126 those of V, 63 is all ones (the row sums).
// The int8 matrix instructions multiply signed bytes: both operands are
// offset by 128 (a byte u is stored as u - 128), and
//   sum a_u b_u = sum a_s b_s + 128 sum_K a_s + 128 sum_K b_u,
// where sum_K a_s is the all-ones column and sum_K b_u follows from the byte
// sums of U and V. Each workgroup takes 128 rows and one chunk of K
// (at most 2^15 bytes: |sum a_s b_s| < 2^29 fits the 32-bit accumulators) and
// stores its partial columns; the epilogue adds the chunks, applies the
// offsets, assembles the 520-bit integer per row and reduces it.
#include <string.h>

#include <algorithm>

#include "gkr_bodies.hpp"
#include "gkr_contract.hpp"
#include "gkr_profile.hpp"
#include "gkr_program.hpp"

namespace gkr {

typedef int I32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kCcCols = 128;        // B columns: two vectors of 63 bands, the ones column, one unused
constexpr uint32_t kCcOnes = 63;         // the all-ones column
constexpr uint32_t kCcRows = 256;        // rows per workgroup (eight waves of two 16-row groups)
constexpr uint32_t kCcThreads = 512;
constexpr uint32_t kCcBlockK = 256;      // K bytes staged in LDS at a time (four 64-byte steps)
constexpr uint32_t kCcLdsStride = 272;   // bytes per staged column: 16 lanes of one read hit distinct banks
constexpr uint32_t kCcMaxChunkK = 1u << 15;

// ST_CC_BUILD: the banded matrix, stored transposed (Bt[col][K], int8 with
// the 128 offset). Thread t: column t >> n, copy c = t & (2^n - 1), 32 bytes.
// p0 U, p1 V, p2 Bt; u0 n; q0 2^n * 128.
__global__ void __launch_bounds__(kBlock) k_cc_build(Step st) {
  const Fr* U = P<const Fr*>(st, 0);
  const Fr* V = P<const Fr*>(st, 1);
  uint8_t* Bt = P<uint8_t*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t K = 32ull << n;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < st.q[0];
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t col = (uint32_t)(t >> n);
    const uint64_t c = t & ((1ull << n) - 1);
    uint32_t out[8];
    if (col == kCcOnes) {
#pragma unroll
      for (int d = 0; d < 8; ++d) out[d] = 0x01010101u;
    } else if (col == kCcCols - 1) {
#pragma unroll
      for (int d = 0; d < 8; ++d) out[d] = 0;
    } else {
      const Fr x = ldf(col < kCcOnes ? U : V, c);
      const int k = (int)(col < kCcOnes ? col : col - 64);
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        uint32_t word = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = k - (4 * d + e);  // byte i of x meets byte j = 4d + e of W
          uint32_t b = 0;
          if (i >= 0 && i < 32) b = (x.v[i >> 2] >> (8 * (i & 3))) & 0xffu;
          word |= ((b - 128u) & 0xffu) << (8 * e);
        }
        out[d] = word;
      }
    }
    GlobalU4* q = (GlobalU4*)(Bt + (uint64_t)col * K + 32 * c);
    q[0] = U32x4{out[0], out[1], out[2], out[3]};
    q[1] = U32x4{out[4], out[5], out[6], out[7]};
  }
}

// ST_CC_BSUM: byte sums BS[v * 32 + i] = sum_c byte i of (v ? V : U)[c]; one
// workgroup per (v, i). p0 U, p1 V, p2 BS; q0 2^n.
__global__ void __launch_bounds__(kBlock) k_cc_bsum(Step st) {
  const uint32_t v = blockIdx.x >> 5, i = blockIdx.x & 31;
  const uint32_t* X = P<const uint32_t*>(st, v);
  uint32_t s = 0;
  for (uint64_t c = threadIdx.x; c < st.q[0]; c += kBlock) s += (X[8 * c + (i >> 2)] >> (8 * (i & 3))) & 0xffu;
  __shared__ uint32_t red[kBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += (uint32_t)__shfl_xor((int)s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    P<uint32_t*>(st, 2)[blockIdx.x] = t;
  }
}

// ST_CC_GEMM: partial column sums of 256 rows over one K chunk. Workgroup b:
// chunk b / row_tiles, rows 256 (b mod row_tiles) ..; wave w takes the
// 16-row groups 2w and 2w + 1 against all eight 16-column groups. Lane l
// holds 16 bytes of row (l mod 16) and of column (l mod 16) at K offset
// 16 (l / 16) of each 64-byte step (the instruction sums the four lane groups),
// and receives rows 4 (l / 16) .. + 3 of column l mod 16.
// p0 W (bytes), p1 Bt, p2 part (int32 [chunk][row][128]); u0 n, u1 row_tiles;
// q0 chunk bytes, q1 rows.
__global__ void __launch_bounds__(kCcThreads) k_cc_gemm(Step st) {
  __shared__ __attribute__((aligned(16))) uint8_t Bs[kCcCols * kCcLdsStride];
  const uint8_t* W = P<const uint8_t*>(st, 0);
  const uint8_t* Bt = P<const uint8_t*>(st, 1);
  int32_t* part = P<int32_t*>(st, 2);
  const uint32_t n = st.u[0], row_tiles = st.u[1];
  const uint64_t K = 32ull << n, Kc = st.q[0], rows = st.q[1];
  const uint32_t chunk = blockIdx.x / row_tiles, rt = blockIdx.x - chunk * row_tiles;
  const uint64_t y0 = (uint64_t)rt * kCcRows, k0 = (uint64_t)chunk * Kc;
  const uint32_t wid = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const uint32_t nblk = (uint32_t)(Kc / kCcBlockK);
  // this thread's share of a staged block: column t / 4, 64 bytes at (t & 3) * 64
  const uint32_t scol = threadIdx.x >> 2, soff = (threadIdx.x & 3) * 64;
  const U32x4* bsrc = (const U32x4*)(Bt + (uint64_t)scol * K + k0 + soff);
  const U32x4* arow[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) arow[h] = (const U32x4*)(W + (y0 + (2 * wid + h) * 16 + r) * K + k0 + 16 * g);
  I32x4 acc[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cg = 0; cg < 8; ++cg) acc[h][cg] = I32x4{0, 0, 0, 0};
  U32x4 bst[4], anext[2][4];
#pragma unroll
  for (int e = 0; e < 4; ++e) bst[e] = bsrc[e];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int s = 0; s < 4; ++s) anext[h][s] = arow[h][4 * s];  // 64-byte steps: 4 U32x4 apart
  for (uint32_t blk = 0; blk < nblk; ++blk) {
    __syncthreads();  // every wave has finished the previous block's LDS reads
#pragma unroll
    for (int e = 0; e < 4; ++e) *(U32x4*)(Bs + scol * kCcLdsStride + soff + 16 * e) = bst[e];
    U32x4 a[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int s = 0; s < 4; ++s) a[h][s] = anext[h][s];
    __syncthreads();
    if (blk + 1 < nblk) {
      const uint64_t adv = (uint64_t)(blk + 1) * (kCcBlockK / 16);
#pragma unroll
      for (int e = 0; e < 4; ++e) bst[e] = bsrc[adv + e];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < 4; ++s) anext[h][s] = arow[h][adv + 4 * s];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int cg = 0; cg < 8; ++cg) {
        const U32x4 bv = *(const U32x4*)(Bs + (cg * 16 + r) * kCcLdsStride + 64 * s + 16 * g);
        const I32x4 bf = I32x4{(int)bv.x, (int)bv.y, (int)bv.z, (int)bv.w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // W's bytes u as signed u - 128: the top bit of every byte flipped
          const I32x4 af = I32x4{(int)(a[h][s].x ^ 0x80808080u), (int)(a[h][s].y ^ 0x80808080u),
                                 (int)(a[h][s].z ^ 0x80808080u), (int)(a[h][s].w ^ 0x80808080u)};
          acc[h][cg] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf, acc[h][cg], 0, 0, 0);
        }
      }
    }
  }
  // rows 4g .. 4g + 3 of each 16-row group, column cg * 16 + r
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cg = 0; cg < 8; ++cg)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t y = y0 + (2 * wid + h) * 16 + 4 * g + e;
        part[((uint64_t)chunk * rows + y) * kCcCols + cg * 16 + r] = acc[h][cg][e];
      }
}

// ST_CC_EPILOGUE: thread (y, v): the chunk sums of row y's 63 band columns of
// vector v and of the ones column, the offsets, the integer sum_k 2^(8k) E_k
// (below 2^520), its top bits folded by 2^508 mod p (w[0..7], plain form),
// then one Montgomery reduction. p0 part, p1 BS, p2 P out, p3 Q out;
// u0 chunks; q0 rows.
__global__ void __launch_bounds__(kBlock) k_cc_epilogue(Step st) {
  const int32_t* part = P<const int32_t*>(st, 0);
  const uint32_t* BS = P<const uint32_t*>(st, 1);
  const uint32_t chunks = st.u[0];
  const uint64_t rows = st.q[0];
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * rows) return;
  const uint64_t y = t >> 1;
  const uint32_t v = (uint32_t)(t & 1);
  // prefix sums of the vector's byte sums: sum_K b_u of band k covers bytes max(0, k-31) .. min(k, 31)
  uint64_t ps[33];
  ps[0] = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) ps[i + 1] = ps[i] + BS[32 * v + i];
  int64_t rs = 0;
  for (uint32_t ch = 0; ch < chunks; ++ch) rs += part[((uint64_t)ch * rows + y) * kCcCols + kCcOnes];
  uint64_t acc[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) acc[i] = 0;
#pragma unroll
  for (int k = 0; k < 63; ++k) {
    int64_t d = 0;
    for (uint32_t ch = 0; ch < chunks; ++ch) d += part[((uint64_t)ch * rows + y) * kCcCols + 64 * v + k];
    const uint64_t cs = ps[k < 31 ? k + 1 : 32] - ps[k > 31 ? k - 31 : 0];
    const uint64_t e = (uint64_t)(d + 128 * rs + 128 * (int64_t)cs);  // E_k, below 2^33
    const uint64_t sh = e << (8 * (k & 3));                          // below 2^57
    acc[k >> 2] += sh & 0xffffffffu;
    acc[(k >> 2) + 1] += sh >> 32;
  }
  uint32_t lim[17];
  uint64_t carry = 0;
#pragma unroll
  for (int i = 0; i < 17; ++i) {
    const uint64_t s = acc[i] + carry;
    lim[i] = (uint32_t)s;
    carry = s >> 32;
  }
  // fold: S = H 2^508 + L  ==  L + H (2^508 mod p)
  const uint32_t H = (lim[15] >> 28) | (lim[16] << 4);
  lim[15] &= 0x0fffffffu;
  FrWide T;
  uint64_t c2 = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint64_t s = (uint64_t)lim[i] + (i < 8 ? (uint64_t)H * st.w[i] : 0) + c2;
    T.w[i] = (uint32_t)s;
    c2 = s >> 32;
  }
  const Fr out = frw_reduce<4>(T);
  stf(P<Fr*>(st, 2 + v), y, out);
}

void launch_cc_step(const Step& st, hipStream_t s) {
  const int tok = prof_begin(s);
  const dim3 grid(st.ntiles), block(kBlock);
  switch (st.type) {
    case ST_CC_BUILD: k_cc_build<<<grid, block, 0, s>>>(st); break;
    case ST_CC_BSUM: k_cc_bsum<<<grid, block, 0, s>>>(st); break;
    case ST_CC_GEMM: k_cc_gemm<<<grid, dim3(kCcThreads), 0, s>>>(st); break;
    case ST_CC_EPILOGUE: k_cc_epilogue<<<grid, block, 0, s>>>(st); break;
    default: break;
  }
  if (tok >= 0) prof_end(tok, s, PC_COPY_CONTRACT, st.bytes, st.mulmods);
}

// ---------------------------------------------------------------- host

bool cc_applies(uint32_t n, uint32_t sigma) { return n >= kCcMinLogCopies && sigma >= kCcMinLogRows; }

CcPlan cc_plan(uint32_t n, uint32_t sigma) {
  CcPlan cp;
  const uint64_t K = 32ull << n, rows = 1ull << sigma, row_tiles = rows / kCcRows;
  uint64_t chunks = (kCcTargetGroups + row_tiles - 1) / row_tiles;
  chunks = std::max<uint64_t>(chunks, K / kCcMaxChunkK);
  chunks = std::min<uint64_t>(chunks, K / kCcBlockK);
  uint64_t p2 = 1;
  while (p2 < chunks) p2 *= 2;
  cp.chunks = (uint32_t)p2;
  cp.chunk_bytes = K / p2;
  cp.row_tiles = (uint32_t)row_tiles;
  cp.bt_bytes = (size_t)kCcCols * K;
  cp.part_bytes = (size_t)p2 * rows * kCcCols * sizeof(int32_t);
  cp.bs_bytes = 64 * sizeof(uint32_t);
  return cp;
}

size_t cc_scratch_bytes(uint32_t n, uint32_t sigma) {
  if (!cc_applies(n, sigma)) return 0;
  const CcPlan cp = cc_plan(n, sigma);
  return cp.bt_bytes + cp.part_bytes + 256;
}

// 2^508 mod p in plain form: (2^508 R) R^-1 from Montgomery powers of 2.
static void two_pow_508(uint32_t out[8]) {
  const Fr two = fr_to_mont(fr_make(2, 0, 0, 0, 0, 0, 0, 0));
  Fr acc = fr_to_mont(fr_make(1, 0, 0, 0, 0, 0, 0, 0));
  for (int i = 0; i < 508; ++i) acc = fr_mul(acc, two);
  const Fr plain = fr_from_mont(acc);
  for (int k = 0; k < 8; ++k) out[k] = plain.v[k];
}

void emit_copy_contract_mfma(Program& pg, const Fr* W, const Fr* U, const Fr* V, Fr* Pt, Fr* Qt, uint32_t n,
                             uint32_t sigma, void* scratch) {
  const CcPlan cp = cc_plan(n, sigma);
  uint8_t* base = static_cast<uint8_t*>(scratch);
  uint8_t* Bt = base;
  int32_t* part = reinterpret_cast<int32_t*>(base + cp.bt_bytes);
  uint32_t* BS = reinterpret_cast<uint32_t*>(base + cp.bt_bytes + cp.part_bytes);
  const uint64_t rows = 1ull << sigma, ncop = 1ull << n;
  auto mk = [](uint32_t type, uint32_t tiles) {
    Step st;
    memset(&st, 0, sizeof(st));
    st.type = type;
    st.ntiles = tiles < 1 ? 1 : tiles;
    return st;
  };
  {
    const uint64_t t = ncop * kCcCols;
    Step st = mk(ST_CC_BUILD, (uint32_t)std::min<uint64_t>((t + kBlock - 1) / kBlock, 65535u * 8));
    st.p[0] = U; st.p[1] = V; st.p[2] = Bt; st.u[0] = n; st.q[0] = t;
    st.bytes = 64.0 * ncop + (double)cp.bt_bytes;
    pg.steps.push_back(st);
  }
  {
    Step st = mk(ST_CC_BSUM, 64);
    st.p[0] = U; st.p[1] = V; st.p[2] = BS; st.q[0] = ncop;
    st.bytes = 64.0 * ncop;
    pg.steps.push_back(st);
  }
  {
    Step st = mk(ST_CC_GEMM, cp.row_tiles * cp.chunks);
    st.p[0] = W; st.p[1] = Bt; st.p[2] = part; st.u[0] = n; st.u[1] = cp.row_tiles;
    st.q[0] = cp.chunk_bytes; st.q[1] = rows;
    st.bytes = 32.0 * (double)(rows << n) + (double)cp.part_bytes;  // no field products: int8 matrix work
    pg.steps.push_back(st);
  }
  {
    Step st = mk(ST_CC_EPILOGUE, (uint32_t)((2 * rows + kBlock - 1) / kBlock));
    st.p[0] = part; st.p[1] = BS; st.p[2] = Pt; st.p[3] = Qt; st.u[0] = cp.chunks; st.q[0] = rows;
    two_pow_508(st.w);
    st.bytes = (double)cp.part_bytes + 64.0 * rows;
    st.mulmods = (double)rows;  // one reduction per row and vector
    pg.steps.push_back(st);
  }
}

}  // namespace gkr
