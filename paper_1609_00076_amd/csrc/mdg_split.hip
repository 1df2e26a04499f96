// mdg_split.hip -- FP64-accurate GEMM emulated on the INT8 matrix cores (Ozaki scheme).
//
// C := alpha*op(A)*op(B) + beta*C (the dgemm operation of the paper, section 1.2) computed as:
//   1. scale every row i of op(A) by 2^-e_i and every column j of op(B) by 2^-f_j, where e_i (f_j)
//      is the binary exponent of the row's (column's) largest magnitude, so scaled entries lie in
//      (-1, 1) (Ozaki, Ogita, Oishi, Rump, Numer. Algorithms 2012; Ootomo, Ozaki, Yokota, IJHPCA
//      2024);
//   2. split each scaled entry x into S int8 slices q_1..q_S, x = sum_s q_s 2^-7s + r 2^-7S,
//      by S exact binary64 steps (x := 128x, q := trunc(x), x := x - q);
//   3. form the slice products P_st = A_s B_t with s + t <= S + 1 exactly in INT32, summed per
//      anti-diagonal d = s + t: up to 8 slices on v_mfma_i32_32x32x32_i8 (128x64 tiles, 32-deep
//      k-steps), for 9 and 10 slices on v_mfma_i32_16x16x64_i8 (64x64 tiles, 64-deep k-steps);
//   4. recombine in binary64: C' = sum_d 2^-7d sum_{s+t=d} P_st, unscale by 2^(e_i + f_j), and
//      apply alpha and beta in binary64.
// A row of op(A) or column of op(B) holding NaN or Inf is flagged by the exponent pass, and the
// epilogue writes NaN to its row or column of C (the product there is not finite).
// Slices live in a workspace (the caller's, or the library's static scratch array for the
// no-allocation entry point) as 32-deep k-panels of 1 KiB chunks of 32 rows (slice_offset), padded
// with zeros to multiples of 128 rows and 64 k-values.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <type_traits>

#include <cstdint>

#include "mdg.h"
#include "mdg_internal.h"

namespace mdg_split_impl {

constexpr int kBeta = 7;          // bits per slice
constexpr int kKStep = 64;        // k per INT8 MFMA (and per LDS stage)
constexpr int kMaxSlices = 10;    // double-buffered LDS stage of 64x64 tiles fits up to here
constexpr int kSliceMax = 127;    // |q| bound
constexpr int kBufferWord3 = 0x00020000;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const uint32_t num = bytes <= 0 ? 0u : bytes >= (int64_t)0xFFFFFFFF ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)num, kBufferWord3);
}

// ------------------------------------------------------------------------------------------------
// Slicing. X is a rows x k matrix given by its storage: x(r,p) = X[r*ld + p] when ROW_CONTIG
// (op(A) with transa = T, op(B)^T with transb = N), else X[p*ld + r]. Output: exps[r] and the
// slices in k-panel tiles: byte (s, r, p) at slice_offset(s, r, p) for r < rp (rows rounded up
// to 128) and p < kp (k rounded up to 64), zero for r >= rows or p >= k. Within slice s, the
// 32 k-values p = 32c .. 32c+31 of all rp rows form panel c (rp * 32 bytes); the panel holds
// 1 KiB chunks of 32 consecutive rows, and in a chunk row i keeps its two 16-byte halves h at
// 16-byte slots row_slot(i, h). A chunk is what one wave moves into LDS with one direct load, and
// the slot order makes the fragment reads of 8 or 16 consecutive rows hit distinct LDS banks.
// ------------------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }
__host__ __device__ __forceinline__ int64_t round128(int64_t x) { return (x + 127) / 128 * 128; }

__host__ __device__ __forceinline__ int row_slot(int i, int h) {  // i in 0..31, h in 0..1
  return 2 * i + (h ^ (((i >> 2) ^ (i >> 3)) & 1));
}

__device__ __forceinline__ int64_t slice_offset(int s, int64_t r, int64_t p, int64_t rp,
                                                int64_t kp) {
  return (int64_t)s * rp * kp + (p >> 5) * rp * 32 + (r >> 5) * 1024 +
         16 * row_slot((int)(r & 31), (int)((p >> 4) & 1)) + (p & 15);
}
__device__ __forceinline__ int row_exponent(double mx) {
  int e = 0;
  if (mx != 0.0) (void)frexp(mx, &e);  // mx = f * 2^e, f in [0.5, 1)
  return e;
}

// Slices of 16 consecutive entries (already scaled into (-1, 1)) to S 16-byte groups.
template <int S>
__device__ __forceinline__ void slice16(double (&v)[16], v4i (&q)[S]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      v[e] *= (double)(1 << kBeta);
      const double t = trunc(v[e]);
      v[e] -= t;
      w[e / 4] |= ((uint32_t)(int)t & 0xFFu) << (8 * (e % 4));
    }
    q[s] = (v4i){(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
  }
}

// Exponents are gathered in two passes. Pass 1 (split_max_kernel) takes the maximum magnitude of
// each row over a chunk of k and merges the chunks with an integer atomicMax on the encoded
// exponent enc = e + kExpBias (frexp's exponent is monotonic in the magnitude; 0 = no non-zero
// entry yet, so the array starts zeroed). Pass 2 (split_tile_kernel) decodes it.
constexpr int kExpBias = 2048;  // above the magnitude of any binary64 exponent
constexpr int kMaxChunk = 512;  // k per workgroup in pass 1

// A row (column) holding NaN or Inf is marked by kNonFinite, which exceeds every encoded
// exponent, so the atomic maximum keeps it; the exponent-only entry point reports it as
// kNonFiniteExp.
constexpr int kNonFinite = 4 * kExpBias;
constexpr int kNonFiniteExp = 0x7FFFFFFF;

__device__ __forceinline__ int decode_exponent(int enc) { return enc ? enc - kExpBias : 0; }

// Magnitude for the row maximum: NaN and Inf count as Inf (fmax alone would skip a NaN).
__device__ __forceinline__ double max_key(double x) {
  const double a = fabs(x);
  return a <= 1.7976931348623157e308 ? a : __builtin_inf();
}

// alpha-free recombined product of row i and column j: cf * 2^(e_i + f_j), or NaN when either
// operand line holds a non-finite entry.
__device__ __forceinline__ double unscale(double cf, int enc_a, int enc_b) {
  if (enc_a == kNonFinite || enc_b == kNonFinite) return __builtin_nan("");
  return ldexp(cf, decode_exponent(enc_a) + decode_exponent(enc_b));
}

__global__ void __launch_bounds__(256) zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

__global__ void __launch_bounds__(256) decode_exponents_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = p[i] == kNonFinite ? kNonFiniteExp : decode_exponent(p[i]);
}

// Pass 1 over a 64-row block and a kMaxChunk-deep chunk of k; one thread per row (of the 64),
// four k-phases. ROW_CONTIG: x(r,p) = X[r*ld + p]; else X[p*ld + r] (64 lanes read 512
// contiguous bytes of one column).
template <bool ROW_CONTIG>
__global__ void __launch_bounds__(256) split_max_kernel(const double* X, int64_t ld, int64_t rows,
                                                        int64_t k, int32_t* enc) {
  __shared__ double red[4][64];
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * 64, p0 = (int64_t)blockIdx.y * kMaxChunk;
  const int64_t p1 = p0 + kMaxChunk < k ? p0 + kMaxChunk : k;
  double mx = 0.0;
  if (!ROW_CONTIG) {
    const int r = t & 63;
    if (row0 + r < rows)
      for (int64_t p = p0 + (t >> 6); p < p1; p += 4) mx = fmax(mx, max_key(X[p * ld + row0 + r]));
    red[t >> 6][r] = mx;
  } else {
    // wave w takes rows w, w+4, ...; its lanes read 64 consecutive k of a row
    const int lane = t & 63, w = t >> 6;
    for (int rr = w; rr < 64; rr += 4) {
      double m2 = 0.0;
      if (row0 + rr < rows)
        for (int64_t p = p0 + lane; p < p1; p += 64) m2 = fmax(m2, max_key(X[(row0 + rr) * ld + p]));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m2 = fmax(m2, __shfl_xor(m2, off, 64));
      if (lane == 0) red[0][rr] = m2;
    }
    if (t < 64) { red[1][t] = 0.0; red[2][t] = 0.0; red[3][t] = 0.0; }
  }
  __syncthreads();
  if (t < 64 && row0 + t < rows) {
    const double m = fmax(fmax(red[0][t], red[1][t]), fmax(red[2][t], red[3][t]));
    if (m != 0.0)
      atomicMax(enc + row0 + t, m == __builtin_inf() ? kNonFinite : row_exponent(m) + kExpBias);
  }
}

// Pass 2: one 64 x 64 block (rows x k) per workgroup, staged through LDS so that the global reads
// are 512-byte runs for either storage order; thread t then slices row t/4, k-values
// 16*(t%4) .. +15 and writes S 16-byte groups, so a wave writes two 512-byte runs per slice.
// The grid covers rp rows; blocks past the matrix write zero rows.
template <int S, bool ROW_CONTIG>
__global__ void __launch_bounds__(256) split_tile_kernel(const double* X, int64_t ld, int64_t rows,
                                                         int64_t k, int64_t kp, int8_t* out,
                                                         const int32_t* enc) {
  __shared__ double tile[64][65];  // [row][k], one double of padding per row
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * 64, p0 = (int64_t)blockIdx.y * 64;
  const int64_t rp = round128(rows);
  if (!ROW_CONTIG) {
    const int r = t & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int pp = (t >> 6) + 4 * i;
      tile[r][pp] = (row0 + r < rows && p0 + pp < k) ? X[(p0 + pp) * ld + row0 + r] : 0.0;
    }
  } else {
    const int pp = t & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = (t >> 6) + 4 * i;
      tile[r][pp] = (row0 + r < rows && p0 + pp < k) ? X[(row0 + r) * ld + p0 + pp] : 0.0;
    }
  }
  __syncthreads();
  const int r = t >> 2, q0 = 16 * (t & 3);
  const int enc_r = (row0 + r < rows) ? enc[row0 + r] : 0;
  const int e = enc_r == kNonFinite ? 0 : decode_exponent(enc_r);  // such rows' slices are unused
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = ldexp(tile[r][q0 + i], -e);
  v4i q[S];
  slice16<S>(v, q);
#pragma unroll
  for (int s = 0; s < S; ++s)
    *reinterpret_cast<v4i*>(out + slice_offset(s, row0 + r, p0 + q0, rp, kp)) = q[s];
}

// ------------------------------------------------------------------------------------------------
// Slice-product GEMM with FP64 recombination and the alpha/beta epilogue.
//
// Workgroup: 64x64 tile of C. LDS stage per k-step of 64:
// S slices x 64 rows x 64 bytes for each operand. A row's 64 bytes are four 16-byte chunks stored
// in a row-dependent order (see swz), so the rows of one fragment read fall in disjoint banks.
//
// v_mfma_i32_16x16x64_i8(X, Y, Z) gives D = X*Y + Z for a 16x64 X and 64x16 Y; lane l supplies
// the 16 bytes X[l%16][16*(l/16) ..] and Y[16*(l/16) ..][l%16] and holds D[4*(l/16) + r][l%16] in
// accumulator r. With X = B_t^T and Y = A_s^T, D = (A_s B_t)^T and lane l holds
// C(i0 + l%16, j0 + 4*(l/16) + r): 16 consecutive rows of a column per 16 lanes.
// ------------------------------------------------------------------------------------------------
struct SplitArgs {
  int64_t m, n, kp;
  double alpha, beta;
  double* C;
  int64_t ldc;
  const int8_t* As;  // slices of op(A) in k-panel tiles (see slice_offset), rows rounded to 128
  const int8_t* Bs;  // slices of op(B)^T, the same way
  const int32_t* ea;  // encoded exponents (see decode_exponent)
  const int32_t* eb;
  int flush_steps;   // k-steps after which the INT32 accumulators are folded into FP64
};

constexpr int kTile = 64;
constexpr int kStageRow = 64;                         // bytes per row per slice in LDS
constexpr int kSliceBytes = kTile * kStageRow;        // 4 KiB per slice per operand

// The chunk permutation makes the 16-byte reads of 16 consecutive rows at one chunk position
// conflict-free both when the LDS serves 8 lanes per cycle over 32 banks and when it serves 16
// lanes over 64 banks; each row keeps its four chunks, so the staging writes stay conflict-free.
__device__ __forceinline__ int swz(int row, int chunk) {
  return row * kStageRow + ((chunk ^ (((row >> 1) ^ (row >> 3)) & 3)) << 4);
}

// N instructions of class MASK as one scheduling group.
template <int MASK, int N>
__device__ __forceinline__ void sched_group() {
  if constexpr (N > 0) __builtin_amdgcn_sched_group_barrier(MASK, N, 0);
}

// N times: M MFMAs, then one instruction of class MASK (a sched_group_barrier pattern).
template <int MASK, int M, int N>
__device__ __forceinline__ void sched_interleave() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x008, M, 0);
    __builtin_amdgcn_sched_group_barrier(MASK, 1, 0);
    sched_interleave<MASK, M, N - 1>();
  }
}

// 8 waves (2 per SIMD) on a 64x64 tile: wave (wm, wn) with wm in 0..1, wn in 0..3 owns rows
// 32*wm .. +31 (RB = 2 blocks) and columns 16*wn .. +15 (one block). Per k-step a wave holds the S
// B-fragments of its column block and streams the A-fragments slice by slice.
constexpr int kThreads = 512;
constexpr int kRB = 2;

template <int S>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
split_gemm_kernel(SplitArgs g, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(16))) int8_t lds[2][2][S][kSliceBytes];  // [buf][A/B][s][..]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wave_m = wave & 1, wave_n = wave >> 1;
  const int l16 = lane & 15, lq = lane >> 4;

  // Tile order: each XCD gets a contiguous run of tiles, visited in column groups of 8 tile-rows,
  // so the 32 workgroups resident on an XCD cover an 8 x 4 block and share A and B panels in L2.
  // The host rounds the grid up to a multiple of 8; the padding workgroups exit here.
  const int nwg = gridDim.x;
  const int t = (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (t >= tiles_m * tiles_n) return;
  constexpr int kGroup = 8;
  const int per_group = kGroup * tiles_n;
  const int grp = t / per_group, first_m = grp * kGroup;
  const int gsize = min(tiles_m - first_m, kGroup);
  const int rem = t - grp * per_group;
  const int tm = first_m + rem % gsize, tn = rem / gsize;
  const int64_t row0 = (int64_t)tm * kTile, col0 = (int64_t)tn * kTile;

  // Global -> LDS staging: threads 0..255 carry A, 256..511 carry B; thread loads row
  // (tid % 256) >> 2, chunk tid & 3 of every slice of its operand.
  // ld_op is uniform within a wave; saying so keeps the buffer descriptor in scalar registers.
  const int ld_op = __builtin_amdgcn_readfirstlane(tid >> 8);
  const int ld_row = (tid & 255) >> 2, ld_chunk = tid & 3;
  // Each operand's slices are k-panel tiles: this thread's 16 bytes of k-step ks of slice s are at
  // s * slice_stride + ks * step_stride + off0, and a wave's 64 loads cover two 512-byte runs
  // (16 rows of one 1 KiB chunk in each of the step's two 32-deep panels).
  const int64_t rp = round128(ld_op ? g.n : g.m);
  const int64_t slice_stride = rp * g.kp, step_stride = rp * kKStep;
  const rsrc_t rsrc = make_rsrc(ld_op ? (const void*)g.Bs : (const void*)g.As, (int64_t)S * slice_stride);
  // k-chunk c of a 64-deep step lies in 32-deep panel c / 2, half c % 2
  const int64_t ld_r = (ld_op ? col0 : row0) + ld_row;
  const int64_t off0 = (ld_chunk >> 1) * rp * 32 + (ld_r >> 5) * 1024 +
                       16 * row_slot((int)(ld_r & 31), ld_chunk & 1);
  const int st_off = swz(ld_row, ld_chunk);

  // Two register sets of staged data: the panel for step ks+2 is loaded while step ks computes,
  // so a load has two k-steps of arithmetic to arrive before it is written to LDS.
  v4i pre0[S], pre1[S];
  auto fetch = [&](v4i (&pre)[S], int64_t ks) {
#pragma unroll
    for (int s = 0; s < S; ++s)
      // Offsets stay below 2^32: the host keeps each operand's slice array under 4 GiB.
      pre[s] = __builtin_amdgcn_raw_buffer_load_b128(
          rsrc, (int)(s * slice_stride + ks * step_stride + off0), 0, 0);
  };
  auto stage = [&](const v4i (&pre)[S], int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) *reinterpret_cast<v4i*>(&lds[buf][ld_op][s][st_off]) = pre[s];
  };

  v4i acc[S][kRB];  // [diagonal d - 2][bi]
  d4 cf[kRB];       // recombined FP64 sums
#pragma unroll
  for (int bi = 0; bi < kRB; ++bi) {
    cf[bi] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < S; ++d) acc[d][bi] = (v4i){0, 0, 0, 0};
  }

  auto fold = [&]() {
#pragma unroll
    for (int bi = 0; bi < kRB; ++bi)
#pragma unroll
      for (int d = 0; d < S; ++d) {
#pragma unroll
        for (int r = 0; r < 4; ++r) cf[bi][r] += ldexp((double)acc[d][bi][r], -kBeta * (d + 2));
        acc[d][bi] = (v4i){0, 0, 0, 0};
      }
  };

  const int nsteps = (int)(g.kp / kKStep);
  fetch(pre0, 0);
  stage(pre0, 0);
  if (nsteps > 1) fetch(pre1, 1);
  __syncthreads();

  const int a_row = wave_m * 32 + l16;  // fragment rows this lane feeds (plus 16*bi)
  const int b_row = wave_n * 16 + l16;
  int since_fold = 0;

  // One k-step: compute from LDS buffer ks & 1; `next` holds step ks+1 (staged at the end),
  // `spare` receives step ks+2. STEADY: both exist, so the step has no branch around its memory
  // operations (which keeps the compiler's wait counts exact across the loop back edge).
  auto step = [&](auto steady_tag, int ks, v4i (&next)[S], v4i (&spare)[S]) {
    constexpr bool STEADY = decltype(steady_tag)::value;
    const int buf = ks & 1;
    if (STEADY || ks + 2 < nsteps) fetch(spare, (int64_t)(ks + 2));
    // Buffer buf^1 was last read before the previous barrier, so step ks+1 can be staged into
    // it now, while this step's MFMAs run (up to 8 slices; beyond, the registers this keeps
    // live at once would spill, and staging stays at the end of the step).
    constexpr bool kEarly = S <= 8;
    if (kEarly && (STEADY || ks + 1 < nsteps)) stage(next, buf ^ 1);

    v4i bf[S];
#pragma unroll
    for (int s = 0; s < S; ++s) bf[s] = *reinterpret_cast<const v4i*>(&lds[buf][1][s][swz(b_row, lq)]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      v4i af[kRB];
#pragma unroll
      for (int bi = 0; bi < kRB; ++bi)
        af[bi] = *reinterpret_cast<const v4i*>(&lds[buf][0][s][swz(a_row + 16 * bi, lq)]);
#pragma unroll
      for (int tt = 0; tt < S - s; ++tt)  // slice pair (s+1, tt+1): diagonal s + tt + 2
#pragma unroll
        for (int bi = 0; bi < kRB; ++bi)
          acc[s + tt][bi] = __builtin_amdgcn_mfma_i32_16x16x64_i8(bf[tt], af[bi], acc[s + tt][bi], 0, 0, 0);
    }
    if (++since_fold == g.flush_steps) {
      fold();
      since_fold = 0;
    }
    if (!kEarly && (STEADY || ks + 1 < nsteps)) stage(next, buf ^ 1);
    if (kEarly && STEADY) {
      // MFMAs interleaved one by one with this step's global loads, then two by two with the
      // staging writes (0x008 MFMA, 0x020 VMEM read, 0x200 DS write).
      sched_interleave<0x020, 1, S>();
      sched_interleave<0x200, 2, S>();
    }
    __syncthreads();
  };
  using steady_t = std::integral_constant<bool, true>;
  using tail_t = std::integral_constant<bool, false>;
  int ks = 0;
  for (; ks + 3 < nsteps; ks += 2) {
    step(steady_t{}, ks, pre1, pre0);
    step(steady_t{}, ks + 1, pre0, pre1);
  }
  for (; ks < nsteps; ks += 2) {
    step(tail_t{}, ks, pre1, pre0);
    if (ks + 1 < nsteps) step(tail_t{}, ks + 1, pre0, pre1);
  }
  if (since_fold) fold();

  // Epilogue: C(i,j) := alpha * 2^(e_i + f_j) * C'(i,j) + beta * C(i,j).
  const double alpha = g.alpha, beta = g.beta;
#pragma unroll
  for (int bi = 0; bi < kRB; ++bi) {
    const int64_t i = row0 + wave_m * 32 + 16 * bi + l16;
    if (i >= g.m) continue;
    const int enc_i = g.ea[i];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = col0 + wave_n * 16 + 4 * lq + r;
      if (j >= g.n) continue;
      double* c = g.C + j * g.ldc + i;
      const double v = alpha * unscale(cf[bi][r], enc_i, g.eb[j]);
      *c = (beta != 0.0) ? v + beta * *c : v;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Slice-product GEMM on v_mfma_i32_32x32x32_i8, for up to kMaxSlices32 slices.
//
// Workgroup: 128x64 tile of C, 8 waves (2 per SIMD) of 32x32. Per 32-deep k-step the S slices of
// both operands (4 chunks of A and 2 of B per slice, 1 KiB each) go from the workspace straight
// into LDS with direct loads (buffer_load ... lds: lane l's 16 bytes land at the wave-uniform base
// plus 16 l, so a chunk keeps its global byte order, including the row_slot placement). Three LDS
// stages form a ring: the loads for step t+3 go into step t's stage as soon as every wave holds
// all of step t's fragments in registers, so a load has two k-steps to arrive.
//
// v_mfma_i32_32x32x32_i8(X, Y, Z): lane l supplies row l%32 of X (32x32) and column l%32 of Y
// (32x32), 16 k-values each (the same k-order for both, so the product is exact whatever the
// order), and holds D[8*(r/4) + 4*(l/32) + r%4][l%32] in accumulator r (checked on the GPU with an
// in-bounds probe). With X = B_t^T and Y = A_s^T, D = (A_s B_t)^T: lane l holds
// C(i0 + l%32, j0 + 8*(r/4) + 4*(l/32) + r%4), so each accumulator register covers 32 consecutive
// rows of two columns.
// ------------------------------------------------------------------------------------------------
constexpr int kMaxSlices32 = 8;  // 3 stages of 6 KiB x S fit 160 KiB; accumulators fit 256 VGPRs
constexpr int kMT32 = 128, kNT32 = 64, kKStep32 = 32, kChunk = 1024, kStages32 = 3;

template <int S>
struct Cfg32 {
  static constexpr int A_CH = 4 * S, B_CH = 2 * S, CH = A_CH + B_CH;  // chunks per stage
  static constexpr int LOADS = (CH + 7) / 8;  // direct loads per wave per stage (some may be idle)
  static constexpr int STAGE = CH * kChunk;
  static constexpr int TRASH = kStages32 * STAGE;  // 1 KiB that idle loads fill with zeros
  static constexpr int SPLIT = S > 1 ? S / 2 : 1;  // slices multiplied before the mid-step barrier
  static constexpr int HI = S - SPLIT;  // slices multiplied after it
  static constexpr int PART2 = HI * (HI + 1) / 2;  // products after it
  static_assert((kStages32 - 1) * LOADS <= 63, "vmcnt range");
};

typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void* lds_void_ptr;

__device__ __forceinline__ void bare_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// s_waitcnt vmcnt(N) lgkmcnt(0), expcnt untouched. A plain __syncthreads would also wait for the
// direct loads still in flight for later stages.
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N <= 63, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (0 << 8));
}

// The kernel body lives in a device function: the host pass then only sees the kernel's
// signature, and emits its launch stub.
template <int S>
__device__ __forceinline__ void split32_tile(const SplitArgs& g, int tiles_m, int tiles_n,
                                             int8_t* lds) {
  using C = Cfg32<S>;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave_m = wave & 3, wave_n = wave >> 2;

  // Tile order: each XCD gets a contiguous run of tiles, visited in column groups of 4 tile-rows
  // (the 32 workgroups resident on an XCD cover a 4 x 8 block: 512 rows of A, 512 columns of B).
  // The host rounds the grid up to a multiple of 8; the padding workgroups exit here.
  const int nwg = gridDim.x;
  const int t = (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  if (t >= tiles_m * tiles_n) return;
  constexpr int kGroup = 4;
  const int per_group = kGroup * tiles_n;
  const int grp = t / per_group, first_m = grp * kGroup;
  const int gsize = min(tiles_m - first_m, kGroup);
  const int rem = t - grp * per_group;
  const int tm = first_m + rem % gsize, tn = rem / gsize;
  const int64_t row0 = (int64_t)tm * kMT32, col0 = (int64_t)tn * kNT32;

  // Direct loads: load u of wave w moves chunk c = 8u + w of the stage: c < A_CH is chunk c % 4
  // (32 rows) of A slice c / 4, then B's chunks, then idle loads (out of range of an empty buffer,
  // which reads zeros, into the trash chunk). The kind of each load is uniform within the wave.
  const int64_t rpa = round128(g.m), rpb = round128(g.n);
  const int64_t slice_a = rpa * g.kp, slice_b = rpb * g.kp;
  const uint32_t step_a = (uint32_t)(rpa * kKStep32), step_b = (uint32_t)(rpb * kKStep32);
  // Offsets stay below 2^32: the host keeps each operand's slice array under 4 GiB.
  const int64_t bytes_a = (int64_t)S * slice_a, bytes_b = (int64_t)S * slice_b;
  uint32_t voff[C::LOADS];
#pragma unroll
  for (int u = 0; u < C::LOADS; ++u) {
    const int c = 8 * u + wave;
    int64_t o = 0;
    if (c < C::A_CH) o = (c >> 2) * slice_a + (row0 + 32 * (c & 3)) * kKStep32;
    else if (c < C::CH) o = ((c - C::A_CH) >> 1) * slice_b + (col0 + 32 * ((c - C::A_CH) & 1)) * kKStep32;
    voff[u] = (uint32_t)o + 16u * (uint32_t)lane;
  }
  auto issue = [&](int p) __attribute__((always_inline)) {
    int8_t* st = lds + (p % kStages32) * C::STAGE;
#pragma unroll
    for (int u = 0; u < C::LOADS; ++u) {
      const int c = 8 * u + wave;
      const bool is_a = c < C::A_CH, is_b = !is_a && c < C::CH;
      // scalar selects of base, size and k-step; the descriptor is built from them
      const void* base = is_b ? (const void*)g.Bs : (const void*)g.As;
      const int64_t bytes = is_a ? bytes_a : is_b ? bytes_b : 0;
      const uint32_t soff = is_a ? (uint32_t)p * step_a : is_b ? (uint32_t)p * step_b : 0u;
      int8_t* dst = (is_a || is_b) ? st + c * kChunk : lds + C::TRASH;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(make_rsrc(base, bytes), (lds_void_ptr)dst, 16, voff[u],
                                               (int)soff, 0, 0);
    }
  };

  // Fragment reads: lane l reads row l%32 of the wave's chunk, half l/32.
  const int frag = 16 * row_slot(lane & 31, lane >> 5);
  const int a_frag = wave_m * kChunk + frag;                   // + (4 s) KiB
  const int b_frag = (C::A_CH + wave_n) * kChunk + frag;       // + (2 t) KiB
  auto read_a = [&](const int8_t* st, int s) __attribute__((always_inline)) {
    return *reinterpret_cast<const v4i*>(st + a_frag + 4 * s * kChunk);
  };
  v4i bf[S], a0;  // a step's B fragments and its first A fragment, read before the step starts
  auto read_first = [&](const int8_t* st) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < S; ++u) bf[u] = *reinterpret_cast<const v4i*>(st + b_frag + 2 * u * kChunk);
    a0 = read_a(st, 0);
  };

  v16i acc[S];  // [diagonal d - 2]
  double cf[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) cf[r] = 0.0;
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[d][r] = 0;
  auto fold = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cf[r] += ldexp((double)acc[d][r], -kBeta * (d + 2));
        acc[d][r] = 0;
      }
  };
  // slice pairs (s+1, u+1), diagonal s + u + 2
  auto mult = [&](int s, const v4i& a) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < S - s; ++u)
      acc[s + u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[u], a, acc[s + u], 0, 0, 0);
  };

  const int nsteps = (int)(g.kp / kKStep32);  // >= 2: kp is a positive multiple of 64
  const int pre = nsteps < kStages32 ? nsteps : kStages32;
  for (int p = 0; p < pre; ++p) issue(p);
  if (pre == 3) wait_vm_lgkm0<2 * C::LOADS>();
  else wait_vm_lgkm0<C::LOADS>();
  bare_barrier();
  read_first(lds);
  int since_fold = 0;

  // One k-step from stage ts % 3. MID: 0 = the last step (no barrier), 1 = a barrier after the
  // first SPLIT slices with no further loads to issue, 2 = a barrier, then the loads of step
  // ts + 3 into this step's stage (every fragment of this step is in registers by then).
  //   before the barrier: read the A fragments of slices 2..S while slice 1's products run
  //     (B fragments read earliest first), then the products of slices 2..SPLIT;
  //   after it: read the next step's B fragments that the remaining products no longer need and
  //     its first A fragment, issue the loads, run the products of slices SPLIT+1..S, and read the
  //     last B fragments as their final uses retire.
  auto step = [&](auto mid_tag, int ts) __attribute__((always_inline)) {
    constexpr int MID = decltype(mid_tag)::value;
    const int8_t* st = lds + (ts % kStages32) * C::STAGE;
    const int8_t* nst = lds + ((ts + 1) % kStages32) * C::STAGE;
    v4i af[S];
    af[0] = a0;
#pragma unroll
    for (int s = 1; s < S; ++s) af[s] = read_a(st, s);
#pragma unroll
    for (int u = C::HI; u < S; ++u)
      acc[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[u], af[0], acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < C::HI; ++u)
      acc[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[u], af[0], acc[u], 0, 0, 0);
#pragma unroll
    for (int s = 1; s < C::SPLIT; ++s) mult(s, af[s]);
    sched_interleave<0x100, 1, S - 1>();  // one MFMA, one fragment read (0x008 MFMA, 0x100 DS read)
    if constexpr (MID == 2) {
      wait_vm_lgkm0<C::LOADS>();  // step ts + 1 has landed; ts + 2 may be in flight
      bare_barrier();
    } else if constexpr (MID == 1) {
      if (ts + 2 < nsteps) wait_vm_lgkm0<C::LOADS>();
      else wait_vm_lgkm0<0>();
      bare_barrier();
    }
    if constexpr (MID != 0) {
#pragma unroll
      for (int u = C::HI; u < S; ++u) bf[u] = *reinterpret_cast<const v4i*>(nst + b_frag + 2 * u * kChunk);
      a0 = read_a(nst, 0);
    }
    if constexpr (MID == 2) issue(ts + 3);
#pragma unroll
    for (int s = C::SPLIT; s < S; ++s) mult(s, af[s]);
    if constexpr (MID != 0) {
#pragma unroll
      for (int u = C::HI - 1; u >= 0; --u)
        bf[u] = *reinterpret_cast<const v4i*>(nst + b_frag + 2 * u * kChunk);
    }
    if constexpr (MID == 2) {
      sched_group<0x100, C::SPLIT + 1>();                        // next B and A fragments
      sched_interleave<0x020, 1, (C::LOADS < C::PART2 ? C::LOADS : C::PART2)>();  // MFMA, load
    }
    if (++since_fold == g.flush_steps) {
      fold();
      since_fold = 0;
    }
  };
  int ts = 0;
  for (; ts + 3 < nsteps; ++ts) step(std::integral_constant<int, 2>{}, ts);
  for (; ts + 1 < nsteps; ++ts) step(std::integral_constant<int, 1>{}, ts);
  step(std::integral_constant<int, 0>{}, ts);
  if (since_fold) fold();

  // Epilogue: C(i,j) := alpha * 2^(e_i + f_j) * C'(i,j) + beta * C(i,j).
  const int64_t i = row0 + 32 * wave_m + (lane & 31);
  if (i >= g.m) return;
  const int enc_i = g.ea[i];
  const double alpha = g.alpha, beta = g.beta;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t j = col0 + 32 * wave_n + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (j >= g.n) continue;
    double* c = g.C + j * g.ldc + i;
    const double v = alpha * unscale(cf[r], enc_i, g.eb[j]);
    *c = (beta != 0.0) ? v + beta * *c : v;
  }
}

template <int S>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
split_gemm32_kernel(SplitArgs g, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[kStages32 * Cfg32<S>::STAGE + kChunk];
  split32_tile<S>(g, tiles_m, tiles_n, lds);
}

// ------------------------------------------------------------------------------------------------
// Split precision by the Chinese remainder theorem (Ozaki scheme II: Ozaki, Uchino, Imamura 2025).
//
//   1. op(A) row i is scaled to integers of w bits, A'(i,p) = trunc(A(i,p) 2^(w - e_i)), e_i the
//      row maximum's exponent as for the slices (|A'| < 2^w); op(B) column j likewise.
//   2. For each of N pairwise coprime moduli m_l <= 256, the symmetric residues a_l = A' mod m_l
//      and b_l = B' mod m_l lie in [-128, 127] and are stored as int8 "slices" in the same k-panel
//      layout as the slices above (slice l = modulus l).
//   3. P_l = a_l b_l is formed exactly in INT32 on v_mfma_i32_32x32x32_i8 (|P_l| <= k 2^14, folded
//      modulo m_l when k would overflow it) and reduced to r_l = P_l mod m_l in [0, m_l).
//   4. X = sum_l r_l W_l mod M, W_l = (M/m_l) ((M/m_l)^-1 mod m_l), M = prod m_l, taken in
//      (-M/2, M/2]: with 4 k 2^(2w) <= M this is the integer (A'B')(i,j) exactly.
//   5. C := alpha RN(X) 2^(e_i + f_j - 2w) + beta C, RN the rounding of the integer X to binary64.
// N products replace the S(S+1)/2 of the slices for the same accuracy.
// ------------------------------------------------------------------------------------------------
constexpr int kMaxModuli = 24;
constexpr int kCrtMaxBits = 72;
constexpr int kLimbs = 7;  // 32-bit limbs of the integers below 2^224 that step 4 forms
__constant__ int c_moduli[kMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211,
                                         199, 197, 193, 191, 181, 179, 173, 167, 163, 157, 151, 149};
constexpr int kModuliHost[kMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211,
                                         199, 197, 193, 191, 181, 179, 173, 167, 163, 157, 151, 149};

// v mod m for 0 <= v < 2^24 and 2 <= m <= 256 (inv = 1/m in float): the float quotient is the true
// one or one less, so one correction each way makes the remainder exact.
__device__ __forceinline__ int mod_small(int v, int m, float inv) {
  int r = v - (int)((float)v * inv) * m;
  r += (r < 0) ? m : 0;
  r -= (r >= m) ? m : 0;
  return r;
}

// 1/m_l rounded to binary64 and binary32, for the quotients below.
__constant__ double c_inv[kMaxModuli] = {
    1.0 / 256, 1.0 / 255, 1.0 / 253, 1.0 / 251, 1.0 / 247, 1.0 / 241, 1.0 / 239, 1.0 / 233,
    1.0 / 229, 1.0 / 227, 1.0 / 223, 1.0 / 211, 1.0 / 199, 1.0 / 197, 1.0 / 193, 1.0 / 191,
    1.0 / 181, 1.0 / 179, 1.0 / 173, 1.0 / 167, 1.0 / 163, 1.0 / 157, 1.0 / 151, 1.0 / 149};
__constant__ float c_finv[kMaxModuli] = {
    1.0f / 256, 1.0f / 255, 1.0f / 253, 1.0f / 251, 1.0f / 247, 1.0f / 241, 1.0f / 239, 1.0f / 233,
    1.0f / 229, 1.0f / 227, 1.0f / 223, 1.0f / 211, 1.0f / 199, 1.0f / 197, 1.0f / 193, 1.0f / 191,
    1.0f / 181, 1.0f / 179, 1.0f / 173, 1.0f / 167, 1.0f / 163, 1.0f / 157, 1.0f / 151, 1.0f / 149};

// Symmetric residues of 16 scaled entries (integers of at most 72 bits held in binary64) for
// modulus l, as 16 int8 bytes in [-(m/2), m - m/2 - 1]. |a| = c 2^t with c < 2^53 an integer (t > 0
// only past 53 bits, where the low bits of a are zero). d = c - rint(c / m) m is formed exactly by
// one fused multiply-add (it is below 2m in magnitude) with the quotient from binary64, which is
// the nearest integer to c / m or next to it; so d is within one m of the symmetric residue of c,
// and after the sign of a one correction either way gives the residue. Past 53 bits, d is first
// brought into [0, m) and multiplied by 2^t mod m.
struct Parts16 {
  double c[16];
  int t[16];
  bool neg[16];
};

__device__ __forceinline__ void split_parts(const double (&a)[16], Parts16& q) {
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const double x = fabs(a[e]);
    int ex = 0;
    (void)frexp(x, &ex);  // x < 2^ex
    const int t = ex > 53 ? ex - 53 : 0;
    q.c[e] = ldexp(x, -t);
    q.t[e] = t;
    q.neg[e] = a[e] < 0.0;
  }
}

__device__ __forceinline__ v4i residues16(const Parts16& q, int l) {
  const int m = c_moduli[l];
  const double dm = (double)m, inv = c_inv[l];
  const float finv = c_finv[l];
  const int lo = -(m / 2), hi = m - m / 2 - 1;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const double c = q.c[e];
    int x = (int)fma(-rint(c * inv), dm, c);
    if (q.t[e]) {  // times 2^t mod m, t < 20: (2^t mod m) by one shift and reduction
      x += (x < 0) ? m : 0;
      x += (x < 0) ? m : 0;
      x -= (x >= m) ? m : 0;
      x -= (x >= m) ? m : 0;
      const int p2 = mod_small(1 << q.t[e], m, finv);
      x = mod_small(x * p2, m, finv);
    }
    if (q.neg[e]) x = -x;
    x += (x < lo) ? m : 0;
    x -= (x > hi) ? m : 0;
    w[e / 4] |= ((uint32_t)x & 0xFFu) << (8 * (e % 4));
  }
  return (v4i){(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
}

// Step 2 for one operand: one 64 x 64 block (rows x k) per workgroup, staged through LDS as for the
// slices; thread t scales row t/4, k-values 16 (t%4) .. +15, and writes their residues for every
// modulus. Rows with a non-finite entry (flagged by the exponent pass) get zero residues.
template <bool ROW_CONTIG>
__global__ void __launch_bounds__(256) crt_residue_kernel(const double* X, int64_t ld, int64_t rows,
                                                          int64_t k, int64_t kp, int nmod, int bits,
                                                          int8_t* out, const int32_t* enc) {
  __shared__ double tile[64][65];
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * 64, p0 = (int64_t)blockIdx.y * 64;
  const int64_t rp = round128(rows);
  if (!ROW_CONTIG) {
    const int r = t & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int pp = (t >> 6) + 4 * i;
      tile[r][pp] = (row0 + r < rows && p0 + pp < k) ? X[(p0 + pp) * ld + row0 + r] : 0.0;
    }
  } else {
    const int pp = t & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = (t >> 6) + 4 * i;
      tile[r][pp] = (row0 + r < rows && p0 + pp < k) ? X[(row0 + r) * ld + p0 + pp] : 0.0;
    }
  }
  __syncthreads();
  const int r = t >> 2, q0 = 16 * (t & 3);
  const int enc_r = (row0 + r < rows) ? enc[row0 + r] : 0;
  const bool finite = enc_r != kNonFinite;
  const int e = finite ? decode_exponent(enc_r) : 0;
  double a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = finite ? trunc(ldexp(tile[r][q0 + i], bits - e)) : 0.0;
  Parts16 q;
  split_parts(a, q);
  for (int l = 0; l < nmod; ++l)
    *reinterpret_cast<v4i*>(out + slice_offset(l, row0 + r, p0 + q0, rp, kp)) =
        residues16(q, l);
}

// Step 3: the modular products. Workgroup: one modulus l and one MT x NT tile of C, 8 waves of
// WM x WN, each (WM/32) x (WN/32) blocks of v_mfma_i32_32x32x32_i8 (lane layout as in
// split32_tile). The k-steps (KH 32-deep panels each) go through a ring of 3 LDS stages filled by
// direct loads two steps ahead. At the end each lane reduces its accumulators modulo m_l and
// writes them, four columns to a 32-bit word, to R_l[(j/4) m + i] (R_l holds m * ceil(n/4)
// words). Workgroups are ordered modulus-major, so each XCD works on one or two moduli at a time
// and their residue slices stay in its L2 and the Infinity Cache.
constexpr int kCrtStages = 3;
template <int MT_, int NT_, int WM_, int WN_, int KH_>
struct CrtCfg {
  static constexpr int MT = MT_, NT = NT_, WM = WM_, WN = WN_, KH = KH_;
  static constexpr int WAVES_M = MT / WM, WAVES_N = NT / WN;
  static_assert(WAVES_M * WAVES_N == kThreads / 64, "8 waves");
  static constexpr int BI = WM / 32, BJ = WN / 32;       // MFMA blocks per wave
  static constexpr int ACH = MT / 32, BCH = NT / 32;     // 1 KiB chunks per 32-deep panel
  static constexpr int KSTEP = 32 * KH;
  static constexpr int CH = KH * (ACH + BCH);            // chunks per stage
  static constexpr int LOADS = (CH + 7) / 8;             // direct loads per wave per stage
  static constexpr int STAGE = CH * kChunk;
  static constexpr int LDS = kCrtStages * STAGE + kChunk;  // + a trash chunk for idle loads
  static_assert((kCrtStages - 1) * LOADS <= 63, "vmcnt range");
};
// The configuration the library runs: 256 x 128 tiles, 8 waves of 64 x 64, 64-deep steps. Larger
// wave tiles, which read fewer LDS bytes per MFMA (256 x 256 with waves of 128 x 64 or 64 x 128,
// 512 x 128 with 128 x 64), and 128 x 256 tiles all measured within 4% of it at 8192^3: the
// products run at the power limit of the INT8 matrix cores, not at an LDS or issue limit.
using CrtRun = CrtCfg<256, 128, 64, 64, 2>;

struct CrtArgs {
  int64_t m, n, kp;
  const int8_t* As;  // residues of op(A), rows rounded to 128 (slice_offset layout)
  const int8_t* Bs;  // residues of op(B)^T
  uint32_t* R;       // product residues
  int nmod;
  int fold_steps;    // k-steps after which the accumulators are reduced modulo m_l
};

template <class K>
__device__ __forceinline__ void crt_gemm_tile(const CrtArgs& g, int tiles_m, int tiles_n,
                                              int8_t* lds) {
  constexpr int KH = K::KH;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave_m = wave % K::WAVES_M, wave_n = wave / K::WAVES_M;

  // XCD-aware order over (modulus, tile): each XCD a contiguous run, modulus-major, tiles in
  // column groups of 4 tile-rows. The host rounds the grid up to a multiple of 8.
  const int nwg = gridDim.x;
  const int v = (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
  const int tiles = tiles_m * tiles_n;
  if (v >= tiles * g.nmod) return;
  // (the integer divisions run on the vector unit; readfirstlane keeps the results scalar)
  const int l = __builtin_amdgcn_readfirstlane(v / tiles), t = v - l * tiles;
  constexpr int kGroup = 4;
  const int per_group = kGroup * tiles_n;
  const int grp = t / per_group, first_m = grp * kGroup;
  const int gsize = min(tiles_m - first_m, kGroup);
  const int rem = t - grp * per_group;
  const int tm = __builtin_amdgcn_readfirstlane(first_m + rem % gsize);
  const int tn = __builtin_amdgcn_readfirstlane(rem / gsize);
  const int64_t row0 = (int64_t)tm * K::MT, col0 = (int64_t)tn * K::NT;
  const int m_l = c_moduli[l];

  const int64_t rpa = round128(g.m), rpb = round128(g.n);
  const int64_t slice_a = rpa * g.kp, slice_b = rpb * g.kp;
  const int8_t* a_base = g.As + l * slice_a;
  const int8_t* b_base = g.Bs + l * slice_b;
  const int nsteps = (int)(g.kp / K::KSTEP);  // >= 1: kp is a positive multiple of 64

  // Direct load u of wave w moves chunk c = 8u + w of the stage: chunk c < ACH KH is rows
  // 32 (c % ACH).. of A in panel c / ACH of the step, c < CH rows 32 (c' % BCH).. of B in panel
  // c' / BCH (c' = c - ACH KH), the rest idle (an empty buffer into the trash chunk). Rows past
  // the rounded row count read the next panel's rows (still inside the slice) or, past the slice,
  // zeros: either way they feed only rows or columns of C that are not stored.
  uint32_t voff[K::LOADS];
#pragma unroll
  for (int u = 0; u < K::LOADS; ++u) {
    const int c = 8 * u + wave;
    int64_t o = 0;
    if (c < K::ACH * KH) o = (c / K::ACH) * rpa * 32 + (row0 + 32 * (c % K::ACH)) * 32;
    else if (c < K::CH) {
      const int cb = c - K::ACH * KH;
      o = (cb / K::BCH) * rpb * 32 + (col0 + 32 * (cb % K::BCH)) * 32;
    }
    voff[u] = (uint32_t)o + 16u * (uint32_t)lane;
  }
  auto issue = [&](int ks) __attribute__((always_inline)) {
    int8_t* st = lds + (ks % kCrtStages) * K::STAGE;
#pragma unroll
    for (int u = 0; u < K::LOADS; ++u) {
      const int c = 8 * u + wave;
      const bool is_a = c < K::ACH * KH, is_b = !is_a && c < K::CH;
      const int8_t* base = is_b ? b_base : a_base;
      const int64_t bytes = is_a ? slice_a : is_b ? slice_b : 0;
      const uint32_t soff = is_a ? (uint32_t)ks * (uint32_t)(rpa * K::KSTEP)
                                 : is_b ? (uint32_t)ks * (uint32_t)(rpb * K::KSTEP) : 0u;
      int8_t* dst = (is_a || is_b) ? st + c * kChunk : lds + kCrtStages * K::STAGE;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(make_rsrc(base, bytes), (lds_void_ptr)dst, 16,
                                               voff[u], (int)soff, 0, 0);
    }
  };

  const int frag = 16 * row_slot(lane & 31, lane >> 5);
  const int a_frag = K::BI * wave_m * kChunk + frag;                   // + (bi + ACH h) KiB
  const int b_frag = (K::ACH * KH + K::BJ * wave_n) * kChunk + frag;  // + (bj + BCH h) KiB
  v4i af[KH][K::BI], bf[KH][K::BJ];
  auto read = [&](int ks) __attribute__((always_inline)) {
    const int8_t* st = lds + (ks % kCrtStages) * K::STAGE;
#pragma unroll
    for (int h = 0; h < KH; ++h) {
#pragma unroll
      for (int b = 0; b < K::BI; ++b)
        af[h][b] = *reinterpret_cast<const v4i*>(st + a_frag + (b + K::ACH * h) * kChunk);
#pragma unroll
      for (int b = 0; b < K::BJ; ++b)
        bf[h][b] = *reinterpret_cast<const v4i*>(st + b_frag + (b + K::BCH * h) * kChunk);
    }
  };

  v16i acc[K::BI][K::BJ];
#pragma unroll
  for (int bi = 0; bi < K::BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < K::BJ; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0;
  // acc := acc mod m_l (in [0, m_l)), exact for |acc| < 2^31 and m_l >= 128: the float quotient
  // is within two of the truth (v rounds to 24 bits, then the product once), so two corrections
  // each way make the remainder exact.
  const float inv = 1.0f / (float)m_l;
  auto reduce = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int bi = 0; bi < K::BI; ++bi)
#pragma unroll
      for (int bj = 0; bj < K::BJ; ++bj)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int vv = acc[bi][bj][r];
          int x = vv - (int)((float)vv * inv) * m_l;
          x += (x < 0) ? m_l : 0;
          x += (x < 0) ? m_l : 0;
          x -= (x >= m_l) ? m_l : 0;
          x -= (x >= m_l) ? m_l : 0;
          acc[bi][bj][r] = x;
        }
  };
  // The step's MFMAs, kept ahead of the wait and barrier that follow them (sched_barrier), so
  // the matrix unit works through them while the wave waits.
  auto mfma = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < KH; ++h)
#pragma unroll
      for (int bi = 0; bi < K::BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < K::BJ; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[h][bj], af[h][bi], acc[bi][bj],
                                                              0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  };

  const int pre = nsteps < kCrtStages ? nsteps : kCrtStages;
  for (int ks = 0; ks < pre; ++ks) issue(ks);
  if (pre == 3) wait_vm_lgkm0<2 * K::LOADS>();
  else if (pre == 2) wait_vm_lgkm0<K::LOADS>();
  else wait_vm_lgkm0<0>();
  bare_barrier();
  read(0);
  // Steady state: the fragments of step ks are in registers. Multiply, wait for step ks + 1's
  // loads, barrier (every wave has read step ks), refill ks's stage with step ks + 3, read ks + 1.
  int ks = 0, since_fold = 0;
  for (; ks + 3 < nsteps; ++ks) {
    mfma();
    wait_vm_lgkm0<K::LOADS>();
    bare_barrier();
    issue(ks + 3);
    read(ks + 1);
    if (++since_fold == g.fold_steps) {  // uniform; only when k exceeds 2^17
      reduce();
      since_fold = 0;
    }
  }
  for (; ks + 1 < nsteps; ++ks) {  // drain: no loads left to issue
    mfma();
    if (ks + 2 < nsteps) wait_vm_lgkm0<K::LOADS>();
    else wait_vm_lgkm0<0>();
    bare_barrier();
    read(ks + 1);
  }
  mfma();
  reduce();

  const int64_t words_n = (g.n + 3) / 4;
  uint32_t* R = g.R + (int64_t)l * g.m * words_n;
#pragma unroll
  for (int bi = 0; bi < K::BI; ++bi) {
    const int64_t i = row0 + K::WM * wave_m + 32 * bi + (lane & 31);
    if (i >= g.m) continue;
#pragma unroll
    for (int bj = 0; bj < K::BJ; ++bj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = col0 + K::WN * wave_n + 32 * bj + 8 * q + 4 * (lane >> 5);
        if (j >= g.n) continue;
        const uint32_t word = (uint32_t)acc[bi][bj][4 * q] |
                              ((uint32_t)acc[bi][bj][4 * q + 1] << 8) |
                              ((uint32_t)acc[bi][bj][4 * q + 2] << 16) |
                              ((uint32_t)acc[bi][bj][4 * q + 3] << 24);
        R[(j >> 2) * g.m + i] = word;
      }
  }
}

template <class K>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
crt_gemm_kernel(CrtArgs g, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[K::LDS];
  crt_gemm_tile<K>(g, tiles_m, tiles_n, lds);
}

// Step 4 and 5 constants, computed on the host for the call's modulus count. Step 4 works in
// 16-bit limbs (little end first), so that a residue times a limb fits 24 bits and a sum over all
// moduli fits 32.
constexpr int kLimbs16 = 2 * kLimbs;
struct CrtConst {
  uint16_t W[kMaxModuli][kLimbs16];  // W_l
  uint16_t M[kLimbs16];
  uint32_t half[kLimbs];             // M / 2, 32-bit limbs
  double Mf;                         // M rounded to binary64
  int nmod, bits;
};

struct CombineArgs {
  int64_t m, n, ldc;
  double alpha, beta;
  double* C;
  const uint32_t* R;
  const int32_t* ea;
  const int32_t* eb;
};

// Steps 4 and 5: one thread per row i and group of four columns 4w .. 4w+3 (threads of a wave
// take consecutive rows, so the residue words and C are read in contiguous runs). L32: 32-bit
// limbs enough for sum_l r_l W_l (the host picks the smallest).
template <int L32>
__global__ void __launch_bounds__(256) crt_combine_kernel(CombineArgs a, CrtConst k) {
  constexpr int L = 2 * L32;  // 16-bit limbs
  const int64_t words_n = (a.n + 3) / 4;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t w = blockIdx.y;
  if (i >= a.m) return;
  // S_c = sum_l r_l W_l for the four columns at once, so each modulus' word of residues and its
  // limbs of W_l (uniform, read through the scalar unit) are loaded once: 24-bit products, at
  // most 24 of them per limb.
  uint32_t sc[4][L];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int t = 0; t < L; ++t) sc[c][t] = 0;
  for (int l = 0; l < k.nmod; ++l) {
    const uint32_t word = a.R[((int64_t)l * words_n + w) * a.m + i];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t r = (word >> (8 * c)) & 0xFFu;
#pragma unroll
      for (int t = 0; t < L; ++t) sc[c][t] += __umul24(r, (uint32_t)k.W[l][t]);
    }
  }
  const int enc_i = a.ea[i];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t j = 4 * w + c;
    if (j >= a.n) break;
    uint32_t (&s)[L] = sc[c];
    uint32_t carry = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const uint32_t v = s[t] + carry;
      s[t] = v & 0xFFFFu;
      carry = v >> 16;
    }
    // q ~ S / M (within one of the truth); X = S - q M, then one correction either way.
    double sf = 0.0;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) sf = sf * 65536.0 + (double)s[t];
    const uint32_t q = (uint32_t)floor(sf / k.Mf);
    uint32_t mc = 0, borrow = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const uint32_t prod = q * (uint32_t)k.M[t] + mc;  // < 2^13 * 2^16 + 2^13
      mc = prod >> 16;
      const uint32_t sub = (prod & 0xFFFFu) + borrow;
      borrow = s[t] < sub ? 1u : 0u;
      s[t] = (s[t] + (borrow << 16) - sub) & 0xFFFFu;
    }
    uint32_t x[L32];
#pragma unroll
    for (int t = 0; t < L32; ++t) x[t] = s[2 * t] | (s[2 * t + 1] << 16);
    uint32_t M32[L32];
#pragma unroll
    for (int t = 0; t < L32; ++t) M32[t] = (uint32_t)k.M[2 * t] | ((uint32_t)k.M[2 * t + 1] << 16);
    auto ge = [&](const uint32_t (&v)[L32], const uint32_t* b) {
      for (int t = L32 - 1; t >= 0; --t)
        if (v[t] != b[t]) return v[t] > b[t];
      return true;
    };
    auto add_to = [&](uint32_t (&v)[L32], const uint32_t* b) {  // v := v + b (mod 2^(32 L32))
      uint64_t cy = 0;
#pragma unroll
      for (int t = 0; t < L32; ++t) {
        const uint64_t u = (uint64_t)v[t] + b[t] + cy;
        v[t] = (uint32_t)u;
        cy = u >> 32;
      }
    };
    auto sub_from = [&](uint32_t (&v)[L32], const uint32_t* b) {  // v := v - b
      uint64_t br = 0;
#pragma unroll
      for (int t = 0; t < L32; ++t) {
        const uint64_t sb = (uint64_t)b[t] + br;
        br = (uint64_t)v[t] < sb ? 1 : 0;
        v[t] = (uint32_t)((uint64_t)v[t] - sb);
      }
    };
    if (borrow) add_to(x, M32);              // q was one too large
    else if (ge(x, M32)) sub_from(x, M32);   // q was one too small
    // Signed representative: X >= M/2 stands for X - M; take its magnitude M - X.
    const bool neg = ge(x, k.half);
    if (neg) {
      uint32_t mm[L32];
#pragma unroll
      for (int t = 0; t < L32; ++t) mm[t] = M32[t];
      sub_from(mm, x);
#pragma unroll
      for (int t = 0; t < L32; ++t) x[t] = mm[t];
    }
    // RN(|X|): the top 64 bits, with a sticky bit for anything below, converted once.
    int top = L32 - 1;
    while (top > 0 && x[top] == 0) --top;
    double mag;
    if (top <= 1) {
      mag = (double)(((uint64_t)(L32 > 1 ? x[1] : 0u) << 32) | x[0]);
    } else {
      const int lz = __builtin_clz(x[top]);  // x[top] != 0 here
      uint64_t hi = ((uint64_t)x[top] << 32) | x[top - 1];
      uint32_t below = x[top - 2];
      hi = lz ? (hi << lz) | (below >> (32 - lz)) : hi;
      below = lz ? below << lz : below;
      bool sticky = below != 0;
      for (int t = top - 3; t >= 0; --t) sticky |= x[t] != 0;
      mag = ldexp((double)(hi | (sticky ? 1u : 0u)), 32 * (top - 1) - lz);
    }
    const double xf = neg ? -mag : mag;
    const int enc_j = a.eb[j];
    double v;
    if (enc_i == kNonFinite || enc_j == kNonFinite) {
      v = __builtin_nan("");
    } else {
      v = ldexp(xf, decode_exponent(enc_i) + decode_exponent(enc_j) - 2 * k.bits);
    }
    double* cp = a.C + j * a.ldc + i;
    v = a.alpha * v;
    *cp = (a.beta != 0.0) ? v + a.beta * *cp : v;
  }
}

typedef void (*SliceFn)(const double*, int64_t, int64_t, int64_t, int64_t, int8_t*,
                        const int32_t*);
typedef void (*GemmFn)(SplitArgs, int, int);

// The GEMM kernel for S slices: the 32x32x32 kernel up to kMaxSlices32 (128x64 tiles, 32-deep
// steps), the 16x16x64 kernel beyond (64x64 tiles, 64-deep steps).
struct Fns {
  SliceFn rows, cols;
  GemmFn gemm;
  int mt, nt, kstep;
};

const Fns kFns[kMaxSlices + 1] = {
    {nullptr, nullptr, nullptr, 0, 0, 0},
    {split_tile_kernel<1, true>, split_tile_kernel<1, false>, split_gemm32_kernel<1>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<2, true>, split_tile_kernel<2, false>, split_gemm32_kernel<2>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<3, true>, split_tile_kernel<3, false>, split_gemm32_kernel<3>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<4, true>, split_tile_kernel<4, false>, split_gemm32_kernel<4>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<5, true>, split_tile_kernel<5, false>, split_gemm32_kernel<5>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<6, true>, split_tile_kernel<6, false>, split_gemm32_kernel<6>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<7, true>, split_tile_kernel<7, false>, split_gemm32_kernel<7>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<8, true>, split_tile_kernel<8, false>, split_gemm32_kernel<8>, kMT32, kNT32, kKStep32},
    {split_tile_kernel<9, true>, split_tile_kernel<9, false>, split_gemm_kernel<9>, kTile, kTile, kKStep},
    {split_tile_kernel<10, true>, split_tile_kernel<10, false>, split_gemm_kernel<10>, kTile, kTile, kKStep},
};
static_assert(kMaxSlices32 == 8 && kMaxSlices == 10, "the table above lists each slice count");

bool is_notrans(char t) { return t == 'N' || t == 'n'; }
bool is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
int64_t max1(int64_t x) { return x > 1 ? x : 1; }
int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }
int64_t kpad(int64_t k) { return (k + kKStep - 1) / kKStep * kKStep; }

struct Layout {
  int64_t kp, a_bytes, b_bytes, ea_off, eb_off, total;
};

Layout layout(int64_t m, int64_t n, int64_t k, int S) {
  Layout L;
  L.kp = kpad(k);
  L.a_bytes = align256((int64_t)S * round128(m) * L.kp);
  L.b_bytes = align256((int64_t)S * round128(n) * L.kp);
  L.ea_off = L.a_bytes + L.b_bytes;
  L.eb_off = L.ea_off + align256(4 * m);
  L.total = L.eb_off + align256(4 * n);
  return L;
}

int launch(const void* fn, dim3 grid, dim3 block, hipStream_t s, void** argv) {
  const hipError_t e = hipLaunchKernel(fn, grid, block, argv, 0, s);
  if (e != hipSuccess) {
    mdg_record_hip_error((int)e);
    return MDG_ERR_HIP;
  }
  return MDG_SUCCESS;
}

// Slices and encoded exponents of one operand; `exps` must hold zeros on entry.
int launch_slices(const Fns& f, bool row_contig, const double* X, int64_t ld, int64_t rows,
                  int64_t k, int64_t kp, int8_t* out, int32_t* exps, hipStream_t s) {
  if (rows == 0) return MDG_SUCCESS;
  const unsigned max_blocks = (unsigned)(round64(rows) / 64);
  const unsigned row_blocks = (unsigned)(round128(rows) / 64);
  if (k > 0) {
    void* argv[] = {&X, &ld, &rows, &k, &exps};
    const dim3 grid(max_blocks, (unsigned)((k + kMaxChunk - 1) / kMaxChunk));
    const void* fn = row_contig ? reinterpret_cast<const void*>(&split_max_kernel<true>)
                                : reinterpret_cast<const void*>(&split_max_kernel<false>);
    const int st = launch(fn, grid, dim3(256), s, argv);
    if (st) return st;
  }
  if (kp == 0) return MDG_SUCCESS;  // k = 0: no slices; every exponent stays 0
  void* argv[] = {&X, &ld, &rows, &k, &kp, &out, &exps};
  return launch(reinterpret_cast<const void*>(row_contig ? f.rows : f.cols),
                dim3(row_blocks, (unsigned)(kp / kKStep)), dim3(256), s, argv);
}

int launch_fill(const void* fn, int32_t* p, int64_t n, hipStream_t s) {
  if (n == 0) return MDG_SUCCESS;
  void* argv[] = {&p, &n};
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  return launch(fn, dim3((unsigned)blocks), dim3(256), s, argv);
}

// Checks of the split entry points' arguments 1-14, in dgemm order (the slice count is 14).
int split_check(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                const double* C, int64_t ldc, int nslices) {
  if (!is_notrans(transa) && !is_trans(transa)) return 1;
  if (!is_notrans(transb) && !is_trans(transb)) return 2;
  if (m < 0) return 3;
  if (n < 0) return 4;
  if (k < 0) return 5;
  const bool empty = (m == 0 || n == 0);
  const bool no_product = (alpha == 0.0 || k == 0);
  const bool reads_ab = !empty && !no_product;
  const int64_t rows_a = is_notrans(transa) ? m : k;
  const int64_t rows_b = is_notrans(transb) ? k : n;
  if (reads_ab && A == nullptr) return 7;
  if (lda < max1(rows_a)) return 8;
  if (reads_ab && B == nullptr) return 9;
  if (ldb < max1(rows_b)) return 10;
  if (!empty && !(no_product && beta == 1.0) && C == nullptr) return 12;
  if (ldc < max1(m)) return 13;
  if (nslices < 1 || nslices > kMaxSlices) return 14;
  return MDG_SUCCESS;
}

// Limits of one launch: slice offsets are 32-bit, and the tile count must fit the grid.
int split_size_check(int64_t m, int64_t n, int nslices, const Layout& L) {
  if (L.a_bytes > (int64_t)0xFFFFFFFF - 4096 || L.b_bytes > (int64_t)0xFFFFFFFF - 4096)
    return MDG_ERR_SIZE;
  const Fns& f = kFns[nslices];
  const int64_t tiles_m = (m + f.mt - 1) / f.mt, tiles_n = (n + f.nt - 1) / f.nt;
  if (tiles_m * tiles_n > (int64_t)INT32_MAX / 256) return MDG_ERR_SIZE;
  return MDG_SUCCESS;
}

// The whole split computation on checked arguments, with the workspace `ws` laid out as L. Clears
// the exponent arrays with a kernel (no memset), then slices both operands and runs the GEMM.
int split_run(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, int nslices, int8_t* ws, const Layout& L, hipStream_t s) {
  const Fns& f = kFns[nslices];
  const int64_t tiles_m = (m + f.mt - 1) / f.mt, tiles_n = (n + f.nt - 1) / f.nt;
  int8_t* as = ws;
  int8_t* bs = ws + L.a_bytes;
  int32_t* ea = reinterpret_cast<int32_t*>(ws + L.ea_off);
  int32_t* eb = reinterpret_cast<int32_t*>(ws + L.eb_off);
  // ea and eb are adjacent: zero both encoded exponent arrays in one launch
  int st = launch_fill(reinterpret_cast<const void*>(&zero_i32_kernel), ea,
                       (L.total - L.ea_off) / 4, s);
  if (st) return st;
  st = launch_slices(f, is_trans(transa), A, lda, m, k, L.kp, as, ea, s);
  if (st) return st;
  st = launch_slices(f, is_notrans(transb), B, ldb, n, k, L.kp, bs, eb, s);
  if (st) return st;

  // INT32 headroom: a diagonal sums at most nslices products of f.kstep terms of magnitude
  // <= 127^2 per k-step.
  const int64_t per_step = (int64_t)nslices * f.kstep * kSliceMax * kSliceMax;
  int flush = (int)((int64_t)INT32_MAX / per_step);
  if (flush < 1) flush = 1;
  SplitArgs g{m, n, L.kp, alpha, beta, C, ldc, as, bs, ea, eb, flush};
  int tm = (int)tiles_m, tn = (int)tiles_n;
  void* argv[] = {&g, &tm, &tn};
  return launch(reinterpret_cast<const void*>(f.gemm), dim3((unsigned)((tiles_m * tiles_n + 7) / 8 * 8)),
                dim3(kThreads), s, argv);  // both GEMM kernels run kThreads threads
}

// ---- Chinese remainder split: host side ----------------------------------------------------------

// Unsigned integers of kLimbs 32-bit limbs (little end first), enough for the modulus products.
struct Big {
  uint32_t d[kLimbs] = {0, 0, 0, 0, 0, 0, 0};
};

Big big_mul_small(const Big& a, uint32_t s) {
  Big r;
  uint64_t c = 0;
  for (int t = 0; t < kLimbs; ++t) {
    const uint64_t v = (uint64_t)a.d[t] * s + c;
    r.d[t] = (uint32_t)v;
    c = v >> 32;
  }
  return r;
}

Big big_div_small(const Big& a, uint32_t s, uint32_t* rem) {
  Big r;
  uint64_t c = 0;
  for (int t = kLimbs - 1; t >= 0; --t) {
    const uint64_t v = (c << 32) | a.d[t];
    r.d[t] = (uint32_t)(v / s);
    c = v % s;
  }
  if (rem) *rem = (uint32_t)c;
  return r;
}

// a >= (v << sh) for v < 2^64
bool big_ge_shifted(const Big& a, uint64_t v, int sh) {
  Big b;
  const int limb = sh / 32, bit = sh % 32;
  const unsigned __int128 x = (unsigned __int128)v << bit;
  for (int t = 0; t < 4; ++t)
    if (limb + t < kLimbs) b.d[limb + t] = (uint32_t)(x >> (32 * t));
    else if ((uint32_t)(x >> (32 * t)) != 0) return false;  // beyond the limbs: b > a
  for (int t = kLimbs - 1; t >= 0; --t)
    if (a.d[t] != b.d[t]) return a.d[t] > b.d[t];
  return true;
}

int inverse_mod(int a, int m) {  // a^-1 mod m for gcd(a, m) = 1
  int t0 = 0, t1 = 1, r0 = m, r1 = a % m;
  while (r1) {
    const int q = r0 / r1;
    int tmp = r0 - q * r1; r0 = r1; r1 = tmp;
    tmp = t0 - q * t1; t0 = t1; t1 = tmp;
  }
  return t0 < 0 ? t0 + m : t0;
}

Big crt_modulus_big(int nmod) {
  Big M;
  M.d[0] = 1;
  for (int l = 0; l < nmod; ++l) M = big_mul_small(M, (uint32_t)kModuliHost[l]);
  return M;
}

// The largest w <= kCrtMaxBits with 4 k 2^(2w) <= M (0 if none): every |A'B'| < M/2 then.
int crt_bits_for(int64_t k, int nmod) {
  if (nmod < 1 || nmod > kMaxModuli || k < 0) return 0;
  const Big M = crt_modulus_big(nmod);
  const uint64_t kk = (uint64_t)(k > 1 ? k : 1) * 4u;
  int w = 0;
  while (w < kCrtMaxBits && big_ge_shifted(M, kk, 2 * (w + 1))) ++w;
  return w;
}

// Fills the step 4 constants; returns the number of 32-bit limbs sum_l r_l W_l needs (below
// nmod * 256 * M).
int crt_constants(int nmod, int bits, CrtConst* c) {
  std::memset(c, 0, sizeof(*c));
  const Big M = crt_modulus_big(nmod);
  for (int l = 0; l < nmod; ++l) {
    uint32_t r = 0;
    const int m = kModuliHost[l];
    const Big Ml = big_div_small(M, (uint32_t)m, nullptr);
    big_div_small(Ml, (uint32_t)m, &r);
    const Big W = big_mul_small(Ml, (uint32_t)inverse_mod((int)r, m));
    for (int t = 0; t < kLimbs; ++t) {
      c->W[l][2 * t] = (uint16_t)(W.d[t] & 0xFFFFu);
      c->W[l][2 * t + 1] = (uint16_t)(W.d[t] >> 16);
    }
  }
  const Big half = big_div_small(M, 2u, nullptr);
  double mf = 0.0;
  for (int t = kLimbs - 1; t >= 0; --t) {
    c->M[2 * t] = (uint16_t)(M.d[t] & 0xFFFFu);
    c->M[2 * t + 1] = (uint16_t)(M.d[t] >> 16);
    c->half[t] = half.d[t];
    mf = mf * 4294967296.0 + (double)M.d[t];
  }
  c->Mf = mf;
  c->nmod = nmod;
  c->bits = bits;
  const Big bound = big_mul_small(M, (uint32_t)nmod * 256u);
  int limbs = kLimbs;
  while (limbs > 1 && bound.d[limbs - 1] == 0) --limbs;
  return limbs;
}

struct CrtLayout {
  int64_t kp, a_bytes, b_bytes, r_bytes, ea_off, eb_off, r_off, total;
};

CrtLayout crt_layout(int64_t m, int64_t n, int64_t k, int nmod) {
  CrtLayout L;
  L.kp = kpad(k);
  L.a_bytes = align256((int64_t)nmod * round128(m) * L.kp);
  L.b_bytes = align256((int64_t)nmod * round128(n) * L.kp);
  L.r_bytes = align256((int64_t)nmod * m * ((n + 3) / 4) * 4);
  L.r_off = L.a_bytes + L.b_bytes;
  L.ea_off = L.r_off + L.r_bytes;
  L.eb_off = L.ea_off + align256(4 * m);
  L.total = L.eb_off + align256(4 * n);
  return L;
}

// Exponents (pass 1, into zeroed `exps`) and residues of one operand.
int launch_crt_residues(bool row_contig, const double* X, int64_t ld, int64_t rows, int64_t k,
                        int64_t kp, int nmod, int bits, int8_t* out, int32_t* exps,
                        hipStream_t s) {
  if (rows == 0) return MDG_SUCCESS;
  if (k > 0) {
    void* argv[] = {&X, &ld, &rows, &k, &exps};
    const dim3 grid((unsigned)(round64(rows) / 64), (unsigned)((k + kMaxChunk - 1) / kMaxChunk));
    const void* fn = row_contig ? reinterpret_cast<const void*>(&split_max_kernel<true>)
                                : reinterpret_cast<const void*>(&split_max_kernel<false>);
    const int st = launch(fn, grid, dim3(256), s, argv);
    if (st) return st;
  }
  if (kp == 0) return MDG_SUCCESS;
  void* argv[] = {&X, &ld, &rows, &k, &kp, &nmod, &bits, &out, &exps};
  const void* fn = row_contig ? reinterpret_cast<const void*>(&crt_residue_kernel<true>)
                              : reinterpret_cast<const void*>(&crt_residue_kernel<false>);
  return launch(fn, dim3((unsigned)(round128(rows) / 64), (unsigned)(kp / 64)), dim3(256), s, argv);
}

int crt_size_check(int64_t m, int64_t n, int nmod, const CrtLayout& L) {
  // per-modulus slices are addressed by 32-bit offsets from a 64-bit base
  if (round128(m) * L.kp > (int64_t)0xFFFFFFFF - 4096 || round128(n) * L.kp > (int64_t)0xFFFFFFFF - 4096)
    return MDG_ERR_SIZE;
  const int64_t tiles = ((m + CrtRun::MT - 1) / CrtRun::MT) * ((n + CrtRun::NT - 1) / CrtRun::NT);
  if (tiles * nmod > (int64_t)INT32_MAX / 256 || (n + 3) / 4 > 65535 || (m + 255) / 256 > INT32_MAX)
    return MDG_ERR_SIZE;
  return MDG_SUCCESS;
}

int crt_run(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
            const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
            int64_t ldc, int nmod, int8_t* ws, const CrtLayout& L, hipStream_t s) {
  const int bits = crt_bits_for(k, nmod);
  int8_t* as = ws;
  int8_t* bs = ws + L.a_bytes;
  uint32_t* R = reinterpret_cast<uint32_t*>(ws + L.r_off);
  int32_t* ea = reinterpret_cast<int32_t*>(ws + L.ea_off);
  int32_t* eb = reinterpret_cast<int32_t*>(ws + L.eb_off);
  int st = launch_fill(reinterpret_cast<const void*>(&zero_i32_kernel), ea,
                       (L.total - L.ea_off) / 4, s);
  if (st) return st;
  st = launch_crt_residues(is_trans(transa), A, lda, m, k, L.kp, nmod, bits, as, ea, s);
  if (st) return st;
  st = launch_crt_residues(is_notrans(transb), B, ldb, n, k, L.kp, nmod, bits, bs, eb, s);
  if (st) return st;
  // INT32 headroom: |a_l b_l| <= 128^2 per term, KSTEP terms per step, plus a residue < 256
  const int fold = (int)(((int64_t)INT32_MAX - 256) / ((int64_t)CrtRun::KSTEP * 128 * 128));
  CrtArgs g{m, n, L.kp, as, bs, R, nmod, fold};
  int tm = (int)((m + CrtRun::MT - 1) / CrtRun::MT), tn = (int)((n + CrtRun::NT - 1) / CrtRun::NT);
  {
    void* argv[] = {&g, &tm, &tn};
    st = launch(reinterpret_cast<const void*>(&crt_gemm_kernel<CrtRun>),
                dim3((unsigned)(((int64_t)tm * tn * nmod + 7) / 8 * 8)), dim3(kThreads), s, argv);
    if (st) return st;
  }
  CrtConst kc;
  const int limbs = crt_constants(nmod, bits, &kc);
  CombineArgs a{m, n, ldc, alpha, beta, C, R, ea, eb};
  void* argv[] = {&a, &kc};
  const void* fn = limbs <= 3   ? reinterpret_cast<const void*>(&crt_combine_kernel<3>)
                   : limbs == 4 ? reinterpret_cast<const void*>(&crt_combine_kernel<4>)
                   : limbs == 5 ? reinterpret_cast<const void*>(&crt_combine_kernel<5>)
                   : limbs == 6 ? reinterpret_cast<const void*>(&crt_combine_kernel<6>)
                                : reinterpret_cast<const void*>(&crt_combine_kernel<7>);
  return launch(fn, dim3((unsigned)((m + 255) / 256), (unsigned)((n + 3) / 4)), dim3(256), s, argv);
}

// ------------------------------------------------------------------------------------------------
// Static scratch for mdg_dgemm_split_noalloc: a file-scope device array, one copy per GPU, held
// until the process ends. Host code never passes the array's name to a kernel (on the host it is
// only a stand-in for the symbol): the device address is looked up once per device with
// hipGetSymbolAddress while that device is current, and kept.
// ------------------------------------------------------------------------------------------------
constexpr int64_t kScratchBytes = (int64_t)64 << 20;
static __device__ __attribute__((aligned(256))) int8_t scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
int8_t* g_scratch_ptr[kMaxScratchDevices];

int scratch_address(int8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    mdg_record_hip_error((int)e);
    return MDG_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxScratchDevices) return MDG_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      mdg_record_hip_error((int)e);
      return MDG_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<int8_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MDG_SUCCESS;
}

}  // namespace mdg_split_impl

using namespace mdg_split_impl;

extern "C" {

int mdg_split_max_slices(void) { return kMaxSlices; }

int64_t mdg_dgemm_split_workspace_size(int64_t m, int64_t n, int64_t k, int nslices) {
  if (m < 0 || n < 0 || k < 0 || nslices < 1 || nslices > kMaxSlices) return -1;
  return layout(m, n, k, nslices).total;
}

int mdg_split_slices(int operand, char trans, int64_t rows, int64_t k, const double* X, int64_t ld,
                     int nslices, int8_t* slices, int32_t* exponents, void* stream) {
  if (operand != 0 && operand != 1) return 1;
  if (!is_notrans(trans) && !is_trans(trans)) return 2;
  if (rows < 0) return 3;
  if (k < 0) return 4;
  // x(r, p) is op(A)(r, p) (operand 0) or op(B)(p, r) (operand 1).
  const bool row_contig = operand == 0 ? is_trans(trans) : is_notrans(trans);
  const int64_t need_ld = row_contig ? k : rows;
  if (rows > 0 && k > 0 && X == nullptr) return 5;
  if (ld < max1(need_ld)) return 6;
  if (nslices < 1 || nslices > kMaxSlices) return 7;
  if (rows > 0 && (slices == nullptr || exponents == nullptr)) return 8;
  if (rows == 0) return MDG_SUCCESS;
  int st = mdg_device_check();
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = launch_fill(reinterpret_cast<const void*>(&zero_i32_kernel), exponents, rows, s);
  if (st) return st;
  st = launch_slices(kFns[nslices], row_contig, X, ld, rows, k, kpad(k), slices, exponents, s);
  if (st) return st;
  return launch_fill(reinterpret_cast<const void*>(&decode_exponents_kernel), exponents, rows, s);
}

int mdg_dgemm_split(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                    double* C, int64_t ldc, int nslices, void* workspace, int64_t workspace_bytes,
                    void* stream) {
  int st = split_check(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nslices);
  if (st) return st;
  const bool no_product = (alpha == 0.0 || k == 0);
  if (m == 0 || n == 0 || (no_product && beta == 1.0)) return MDG_SUCCESS;
  if (no_product)  // C := beta*C needs no slices: the native entry point does exactly this
    return mdg_dgemm(transa, transb, m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc, stream);
  const Layout L = layout(m, n, k, nslices);
  if (workspace == nullptr || workspace_bytes < L.total) return 15;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return 15;
  st = split_size_check(m, n, nslices, L);
  if (st) return st;
  st = mdg_device_check();
  if (st) return st;
  return split_run(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nslices,
                   static_cast<int8_t*>(workspace), L, static_cast<hipStream_t>(stream));
}

int64_t mdg_dgemm_split_noalloc_max_bytes(void) { return kScratchBytes; }

int mdg_dgemm_split_noalloc(char transa, char transb, int64_t m, int64_t n, int64_t k,
                            double alpha, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double beta, double* C, int64_t ldc, int nslices,
                            void* stream) {
  int st = split_check(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nslices);
  if (st) return st;
  const bool no_product = (alpha == 0.0 || k == 0);
  if (m == 0 || n == 0 || (no_product && beta == 1.0)) return MDG_SUCCESS;
  if (no_product)  // no slices and no scratch: the native entry point allocates nothing either
    return mdg_dgemm(transa, transb, m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc, stream);
  const Layout L = layout(m, n, k, nslices);
  if (L.total > kScratchBytes) return MDG_ERR_SCRATCH;
  st = split_size_check(m, n, nslices, L);
  if (st) return st;
  st = mdg_device_check();
  if (st) return st;
  int8_t* ws = nullptr;
  st = scratch_address(&ws);
  if (st) return st;
  return split_run(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nslices, ws, L,
                   static_cast<hipStream_t>(stream));
}

int mdg_crt_max_moduli(void) { return kMaxModuli; }

int mdg_crt_bits(int64_t k, int nmoduli) { return crt_bits_for(k, nmoduli); }

int64_t mdg_dgemm_crt_workspace_size(int64_t m, int64_t n, int64_t k, int nmoduli) {
  if (m < 0 || n < 0 || k < 0 || nmoduli < 1 || nmoduli > kMaxModuli) return -1;
  return crt_layout(m, n, k, nmoduli).total;
}

int mdg_crt_residues(int operand, char trans, int64_t rows, int64_t k, const double* X, int64_t ld,
                     int nmoduli, int bits, int8_t* residues, int32_t* exponents, void* stream) {
  if (operand != 0 && operand != 1) return 1;
  if (!is_notrans(trans) && !is_trans(trans)) return 2;
  if (rows < 0) return 3;
  if (k < 0) return 4;
  const bool row_contig = operand == 0 ? is_trans(trans) : is_notrans(trans);
  if (rows > 0 && k > 0 && X == nullptr) return 5;
  if (ld < max1(row_contig ? k : rows)) return 6;
  if (nmoduli < 1 || nmoduli > kMaxModuli) return 7;
  if (bits < 1 || bits > kCrtMaxBits) return 8;
  if (rows > 0 && (residues == nullptr || exponents == nullptr)) return 9;
  if (rows == 0) return MDG_SUCCESS;
  int st = mdg_device_check();
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = launch_fill(reinterpret_cast<const void*>(&zero_i32_kernel), exponents, rows, s);
  if (st) return st;
  st = launch_crt_residues(row_contig, X, ld, rows, k, kpad(k), nmoduli, bits, residues, exponents,
                           s);
  if (st) return st;
  return launch_fill(reinterpret_cast<const void*>(&decode_exponents_kernel), exponents, rows, s);
}

int mdg_dgemm_crt(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                  double* C, int64_t ldc, int nmoduli, void* workspace, int64_t workspace_bytes,
                  void* stream) {
  if (nmoduli < 1 || nmoduli > kMaxModuli) {
    // report an earlier bad argument first, as for the other entry points
    const int st = split_check(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, 1);
    return st ? st : 14;
  }
  int st = split_check(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, 1);
  if (st) return st;
  const bool no_product = (alpha == 0.0 || k == 0);
  if (m == 0 || n == 0 || (no_product && beta == 1.0)) return MDG_SUCCESS;
  if (no_product)  // C := beta*C needs no residues: the native entry point does exactly this
    return mdg_dgemm(transa, transb, m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc, stream);
  if (crt_bits_for(k, nmoduli) < 1) return 14;  // too few moduli for this k
  const CrtLayout L = crt_layout(m, n, k, nmoduli);
  if (workspace == nullptr || workspace_bytes < L.total) return 15;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return 15;
  st = crt_size_check(m, n, nmoduli, L);
  if (st) return st;
  st = mdg_device_check();
  if (st) return st;
  return crt_run(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nmoduli,
                 static_cast<int8_t*>(workspace), L, static_cast<hipStream_t>(stream));
}

}  // extern "C"
