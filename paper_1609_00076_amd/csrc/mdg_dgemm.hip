// mdg_dgemm.hip -- FP64 GEMM on the MI355X (gfx950) matrix cores, behind the C ABI of include/mdg.h.
//
// Operation (paper, section 1.2): C := alpha*op(A)*op(B) + beta*C, column-major with leading
// dimensions (paper, section 2.3). The paper's blocked algorithm (section 4.1: the five loops
// around a micro-kernel, with packing into contiguous panels) is realised for a GPU as:
//   loops 5 and 3 (jc, ic)   -> the grid: one workgroup per mt x nt macro-tile of C;
//   loop 4 (pc) and packing  -> a loop over kt-deep k-panels; each panel of op(A) (mt x kt) and
//                               op(B) (kt x nt) is staged from HBM into LDS, transposed on the way
//                               when the operand is stored the other way round;
//   loops 2 and 1 (jr, ir)   -> the waves of a workgroup, each owning a wm x wn sub-tile;
//   loop 0 (the micro-kernel)-> chains of v_mfma_f64_16x16x4_f64, each one four rank-1 updates of a
//                               16x16 block held in accumulator registers (section 4.3).
// Fringes (section 2.4: m, n, k not multiples of the block sizes) are handled in the kernel: an
// operand is read through a buffer resource whose byte range is the operand's extent, so a load past
// the end returns zero without touching memory; loads of padding rows or of k beyond the logical
// depth are zeroed (or masked out of the product) by the row and depth masks; stores outside C are
// masked. The padding rows of every operand are thus never used and never written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <vector>
#include <cstdint>
#include <cstring>

#include "mdg.h"
#include "mdg_internal.h"

// Kernels need external linkage so the runtime can resolve them by name at launch; everything
// in this namespace is private to the library all the same (only the extern "C" API is exported).
namespace mdg_impl {

constexpr int kCUs = 256;  // MI355X compute units

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kVersion = 100;  // 0.1.0

struct GemmArgs {
  int64_t m, n, k;
  int64_t lda, ldb, ldc;
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  int64_t ext_a, ext_b;  // storage extent of A and B in elements: (cols-1)*ld + rows
};

// ------------------------------------------------------------------------------------------------
// Tile configuration. MT x NT macro-tile per workgroup, KT-deep k-panels, WM x WN per wave.
// ------------------------------------------------------------------------------------------------
template <int MT_, int NT_, int KT_, int WM_, int WN_, int MIN_WAVES_PER_EU_, int PAD_MODE_ = 1>
struct Cfg {
  static constexpr int MT = MT_, NT = NT_, KT = KT_, WM = WM_, WN = WN_;
  static constexpr int MIN_WAVES_PER_EU = MIN_WAVES_PER_EU_;  // occupancy target per SIMD
  // LDS padding: 0 = two doubles per k-row for both operands; 1 = sixteen doubles (128 bytes)
  // for an operand whose global rows run along m or n, which makes the fragment reads of
  // consecutive k-rows fall in disjoint bank halves.
  static constexpr int PAD_MODE = PAD_MODE_;
  static constexpr int WAVES_M = MT / WM, WAVES_N = NT / WN;
  static constexpr int WAVES = WAVES_M * WAVES_N;
  static constexpr int THREADS = WAVES * 64;
  static constexpr int BM = WM / 16, BN = WN / 16;  // 16x16 MFMA blocks per wave
  static constexpr int A_PER_THREAD = MT * KT / THREADS;
  static constexpr int B_PER_THREAD = KT * NT / THREADS;
  static_assert(MT % WM == 0 && NT % WN == 0, "wave grid");
  static_assert(WM % 16 == 0 && WN % 16 == 0 && KT % 4 == 0, "MFMA shape");
  static_assert((MT * KT) % THREADS == 0 && (KT * NT) % THREADS == 0, "panel split");
  static_assert(THREADS <= 1024, "workgroup size");
};

// LDS panels are k-major: element (row r, k-index q) sits at q*STRIDE + r. An operand whose global
// rows run along k is written down a column (16 lanes, 16 k-rows), so its k-rows are two doubles
// apart in bank space (16-byte shift per row, conflict-free writes); an operand whose global rows
// run along m or n is written along a k-row, so its stride can be chosen for the reads instead.
template <class C, bool TA, bool TB>
struct LdsLayout {
  static constexpr int A = (TA || C::PAD_MODE == 0) ? C::MT + 2 : C::MT + 16;
  static constexpr int B = (!TB || C::PAD_MODE == 0) ? C::NT + 2 : C::NT + 16;
};

// XCD-aware tile order. Consecutive workgroup ids are dealt round-robin to the 8 XCDs, each with
// its own L2; the remap gives each XCD a contiguous run of tiles, and within a run tiles are
// visited in column groups of GROUP tile-rows so that co-resident workgroups share A and B panels.
// The host rounds the grid up to a multiple of 8 (kXcds); returns false for the padding
// workgroups, which then exit at once.
constexpr int kXcds = 8;

template <int GROUP = 8>
__device__ __forceinline__ bool tile_coords(int wg, int nwg, int tiles_m, int tiles_n, int& tm,
                                            int& tn) {
  const int t = (wg % kXcds) * (nwg / kXcds) + wg / kXcds;
  if (t >= tiles_m * tiles_n) return false;
  int per_group = GROUP * tiles_n;
  int g = t / per_group;
  int first_m = g * GROUP;
  int gsize = min(tiles_m - first_m, GROUP);
  int r = t - g * per_group;
  tm = first_m + r % gsize;
  tn = r / gsize;
  return true;
}

// ------------------------------------------------------------------------------------------------
// Global -> register panel loads through buffer resources.
//
// Each k-panel of op(A) (MT x KT) and op(B) (KT x NT) is read through a buffer resource whose base
// is the panel's first element and whose size is the rest of the matrix's storage (its exact
// extent, (cols-1)*ld + rows elements, minus the panel origin). A read beyond the matrix's last
// element returns 0 instead of faulting, so no load needs an address clamp. Rows of op(A) beyond m
// and columns of op(B) beyond n may read other data of the same storage; they only feed rows and
// columns of the tile that are never stored. Entries with k-index >= k must be zero in both
// operands (0 * NaN would poison real results); those beyond the last column of the storage are
// zero by the bound above, and the rest are zeroed explicitly in the last, ragged k-panel.
// ------------------------------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ rsrc_t make_rsrc(const double* base, int64_t rem_elems) {
  // num_records is in bytes and 32 bits wide; beyond 4 GiB the bound cannot bind inside a panel.
  const uint32_t num = rem_elems <= 0 ? 0u
                       : rem_elems >= (int64_t)0x1FFFFFFF ? 0xFFFFFFFFu
                                                          : (uint32_t)(rem_elems * 8);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)num,
                                           kBufferWord3);
}

__device__ __forceinline__ double load_f64(rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}

// Per-thread placement of one operand's panel: element r of this thread sits at row `row[r]`,
// k-index `kq[r]` of the panel, `off[r]` bytes from the panel origin in global memory, and at
// `lds[r]` in the k-major LDS panel (index q*LDS + row).
template <int PER_THREAD>
struct PanelMap {
  uint32_t off[PER_THREAD];
  int lds[PER_THREAD];
  int kq[PER_THREAD];
};

// CONTIG_K: the stored operand is contiguous along k (op(A) with transa = T, op(B) with
// transb = N); otherwise it is contiguous along the panel's rows (m for A, n for B).
template <int ROWS, int KT, int THREADS, int LDS, bool CONTIG_K, int PER_THREAD>
__device__ __forceinline__ void make_map(PanelMap<PER_THREAD>& mp, int tid, int64_t ld) {
#pragma unroll
  for (int r = 0; r < PER_THREAD; ++r) {
    const int e = tid + r * THREADS;
    int i, q;
    if (CONTIG_K) { q = e % KT; i = e / KT; }
    else          { i = e % ROWS; q = e / ROWS; }
    mp.off[r] = (uint32_t)((CONTIG_K ? (q + (int64_t)i * ld) : (i + (int64_t)q * ld)) * 8);
    mp.lds[r] = q * LDS + i;
    mp.kq[r] = q;
  }
}

template <int PER_THREAD>
__device__ __forceinline__ void load_panel(const PanelMap<PER_THREAD>& mp, rsrc_t r,
                                           double (&v)[PER_THREAD]) {
#pragma unroll
  for (int e = 0; e < PER_THREAD; ++e) v[e] = load_f64(r, mp.off[e]);
}

template <int PER_THREAD>
__device__ __forceinline__ void mask_k_tail(const PanelMap<PER_THREAD>& mp, int k_left,
                                            double (&v)[PER_THREAD]) {
#pragma unroll
  for (int e = 0; e < PER_THREAD; ++e) v[e] = mp.kq[e] < k_left ? v[e] : 0.0;
}

template <int PER_THREAD>
__device__ __forceinline__ void store_panel(const PanelMap<PER_THREAD>& mp, double* lds,
                                            const double (&v)[PER_THREAD]) {
#pragma unroll
  for (int e = 0; e < PER_THREAD; ++e) lds[mp.lds[e]] = v[e];
}

// One workgroup computes one MT x NT tile of C.
//
// MFMA operand roles: v_mfma_f64_16x16x4_f64(X, Y, Z) forms D = X*Y + Z for a 16x4 X and a 4x16
// Y, where lane l supplies X[l%16][l/16] and Y[l/16][l%16] and holds D[l/16 + 4r][l%16] in its
// r-th accumulator. Feeding X = op(B)^T and Y = op(A)^T makes D = C^T, so lane l holds
// C(i0 + l%16, j0 + l/16 + 4r): lanes 0..15 of each accumulator register cover 16 consecutive
// rows of one column of C, which makes the epilogue's loads and stores of column-major C
// contiguous 128-byte runs.
// LDS doubles one tile of configuration C with transposes TA, TB needs (two buffers per operand).
template <class C, bool TA, bool TB>
constexpr int tile_lds_doubles() {
  return 2 * C::KT * (LdsLayout<C, TA, TB>::A + LdsLayout<C, TA, TB>::B);
}

// Single GEMMs with k <= kPacedK are bound by the old C streaming through HBM. Their interior
// tiles write C paced when beta != 0: after every second store a wave waits until its stores have
// completed. The waves of a CU then leave the epilogue at staggered times, so that some run their
// MFMA loop while others stream C. Measured on m = n = 8192, beta = 1: k = 64 runs 6% faster back
// to back and 15% faster within the full sweep, k = 16, 32, 128 and 256 the same to 1% faster
// (waiting after every store instead cost 4% at k = 16). The latency-bound tiles of a grouped
// launch do not pace (pacing there measured 15% slower).
constexpr int64_t kPacedK = 256;

// The whole computation of tile (tm, tn) of C by one workgroup; `smem` holds
// tile_lds_doubles<C, TA, TB>() doubles. Shared by the single-GEMM kernels and the grouped one,
// so a GEMM computed in a grouped launch is bitwise the one computed alone with the same tile.
// Ends with a workgroup barrier, so the caller may reuse `smem` right away.
template <class C, bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int tm, int tn, double* smem,
                                          bool paced) {
  using L = LdsLayout<C, TA, TB>;
  double (*As)[C::KT * L::A] = reinterpret_cast<double (*)[C::KT * L::A]>(smem);
  double (*Bs)[C::KT * L::B] = reinterpret_cast<double (*)[C::KT * L::B]>(smem + 2 * C::KT * L::A);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wave_m = wave % C::WAVES_M;
  const int wave_n = wave / C::WAVES_M;
  const int l16 = lane & 15, lq = lane >> 4;

  const int64_t row0 = (int64_t)tm * C::MT;
  const int64_t col0 = (int64_t)tn * C::NT;

  // This lane's outputs: rows i0 + 16*bi, columns j0 + 16*bj + 4*r.
  const int64_t i0 = row0 + wave_m * C::WM + l16;
  const int64_t j0 = col0 + wave_n * C::WN + lq;
  double* const cbase = g.C + j0 * g.ldc + i0;
  const double alpha = g.alpha, beta = g.beta;

  // Old C of this lane's outputs in column block bj (BM x 4 values), all loads issued together.
  auto load_c_block = [&](int bj, double (&dst)[C::BM][4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t dj = 16 * bj + 4 * r;
      const bool col_ok = j0 + dj < g.n;
#pragma unroll
      for (int bi = 0; bi < C::BM; ++bi)
        dst[bi][r] = (col_ok && i0 + 16 * bi < g.m) ? cbase[dj * g.ldc + 16 * bi] : 0.0;
    }
  };

  PanelMap<C::A_PER_THREAD> ma;
  PanelMap<C::B_PER_THREAD> mb;
  make_map<C::MT, C::KT, C::THREADS, L::A, TA>(ma, tid, g.lda);
  make_map<C::NT, C::KT, C::THREADS, L::B, !TB>(mb, tid, g.ldb);

  // Panel origins (elements from the matrix base) and their step per k-panel.
  const int64_t a_org = TA ? row0 * g.lda : row0;
  const int64_t a_step = TA ? (int64_t)C::KT : (int64_t)C::KT * g.lda;
  const int64_t b_org = TB ? col0 : col0 * g.ldb;
  const int64_t b_step = TB ? (int64_t)C::KT * g.ldb : (int64_t)C::KT;

  d4 acc[C::BM][C::BN];
#pragma unroll
  for (int bi = 0; bi < C::BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < C::BN; ++bj) acc[bi][bj] = (d4){0.0, 0.0, 0.0, 0.0};

  double ra[C::A_PER_THREAD], rb[C::B_PER_THREAD];
  // alpha == 0 or k == 0: no product (A and B are not read); the epilogue forms beta*C.
  const int num_k = (g.alpha == 0.0) ? 0 : (int)((g.k + C::KT - 1) / C::KT);
  const int k_left_last = (int)(g.k - (int64_t)(num_k - 1) * C::KT);  // 1..KT

  auto fetch = [&](int kt) {
    const int64_t ao = a_org + kt * a_step, bo = b_org + kt * b_step;
    load_panel(ma, make_rsrc(g.A + ao, g.ext_a - ao), ra);
    load_panel(mb, make_rsrc(g.B + bo, g.ext_b - bo), rb);
  };
  // Panel kt to LDS buffer `buf`; the ragged last panel's k-tail is zeroed here rather than right
  // after its loads, so that the arithmetic of the panel before it does not wait for them.
  auto store = [&](int kt, int buf) {
    if (kt == num_k - 1 && k_left_last < C::KT) {  // uniform branch: ragged last panel only
      mask_k_tail(ma, k_left_last, ra);
      mask_k_tail(mb, k_left_last, rb);
    }
    store_panel(ma, As[buf], ra);
    store_panel(mb, Bs[buf], rb);
  };

  if (num_k > 0) {
    fetch(0);
    store(0, 0);
  }
  __syncthreads();

  const int a_frag = lq * L::A + wave_m * C::WM + l16;  // this lane's A fragment at k-step 0
  const int b_frag = lq * L::B + wave_n * C::WN + l16;

  for (int kt = 0; kt < num_k; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < num_k;
    if (more) fetch(kt + 1);
    const double* as = As[buf] + a_frag;
    const double* bs = Bs[buf] + b_frag;
#pragma unroll
    for (int s = 0; s < C::KT / 4; ++s) {
      double af[C::BM], bf[C::BN];
#pragma unroll
      for (int bi = 0; bi < C::BM; ++bi) af[bi] = as[4 * s * L::A + 16 * bi];
#pragma unroll
      for (int bj = 0; bj < C::BN; ++bj) bf[bj] = bs[4 * s * L::B + 16 * bj];
#pragma unroll
      for (int bi = 0; bi < C::BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < C::BN; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[bj], af[bi], acc[bi][bj], 0, 0, 0);
    }
    if (more) store(kt + 1, buf ^ 1);
    __syncthreads();
  }

  // Epilogue: C(i,j) := alpha*acc + beta*C(i,j), rounded as fma(beta, C, alpha*acc) on every path
  // (a result does not depend on which path its tile takes); with beta == 0 the old C is not
  // read. A tile wholly inside C takes a path with no condition on any load or store (one for
  // beta != 0, one for beta == 0): under per-element conditions the compiler cannot count the
  // memory operations in flight and waits for each store to complete before the next goes out.
  if (row0 + C::MT <= g.m && col0 + C::NT <= g.n) {
    if (beta != 0.0) {
#pragma unroll
      for (int bj = 0; bj < C::BN; ++bj) {
        double cb[C::BM][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int bi = 0; bi < C::BM; ++bi) cb[bi][r] = cbase[(16 * bj + 4 * r) * g.ldc + 16 * bi];
        if (paced) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int bi = 0; bi < C::BM; ++bi) {
              cbase[(16 * bj + 4 * r) * g.ldc + 16 * bi] = fma(beta, cb[bi][r], alpha * acc[bi][bj][r]);
              if ((r * C::BM + bi) % 2 == 1) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int bi = 0; bi < C::BM; ++bi)
              cbase[(16 * bj + 4 * r) * g.ldc + 16 * bi] = fma(beta, cb[bi][r], alpha * acc[bi][bj][r]);
        }
      }
    } else {
#pragma unroll
      for (int bj = 0; bj < C::BN; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int bi = 0; bi < C::BM; ++bi)
            cbase[(16 * bj + 4 * r) * g.ldc + 16 * bi] = alpha * acc[bi][bj][r];
    }
    __syncthreads();
    return;
  }
#pragma unroll
  for (int bj = 0; bj < C::BN; ++bj) {
    double cb[C::BM][4];
    if (beta != 0.0) load_c_block(bj, cb);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t dj = 16 * bj + 4 * r;
      if (j0 + dj >= g.n) continue;
#pragma unroll
      for (int bi = 0; bi < C::BM; ++bi) {
        if (i0 + 16 * bi < g.m) {
          const double v = alpha * acc[bi][bj][r];
          cbase[dj * g.ldc + 16 * bi] = (beta != 0.0) ? fma(beta, cb[bi][r], v) : v;
        }
      }
    }
  }
  __syncthreads();
}

template <class C, bool TA, bool TB>
__global__ void __launch_bounds__(C::THREADS) __attribute__((amdgpu_waves_per_eu(C::MIN_WAVES_PER_EU)))
dgemm_mfma_kernel(GemmArgs g, int tiles_m, int tiles_n) {
  __shared__ double smem[tile_lds_doubles<C, TA, TB>()];
  int tm, tn;
  if (!tile_coords(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn)) return;
  gemm_tile<C, TA, TB>(g, tm, tn, smem, g.k <= kPacedK);
}

// C := beta*C over the logical m x n matrix (beta == 0 writes zeros without reading C). This is
// the whole operation when alpha == 0 or k == 0.
__global__ void __launch_bounds__(256) scale_c_kernel(int64_t m, int64_t n, double beta, double* C,
                                                      int64_t ldc) {
  const int64_t total = m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = e / m, i = e - j * m;
    double* c = C + j * ldc + i;
    *c = (beta == 0.0) ? 0.0 : beta * *c;
  }
}

// ------------------------------------------------------------------------------------------------
// Thin products: C blocks with at most kThinMax rows (or columns). Such a block needs the whole of
// the other operand, read once from HBM, and a few multiply-adds per value read, so it is a
// streaming kernel on the vector FMA units rather than MFMA tiles padded to 32 or more rows
// (section 2.4's fringes taken out of the tiled product: see the plan in mdg_dgemm_ex). One form
// covers both orientations:
//   Out(i, l) := alpha * sum_q Y(i, q) X(q, l) + beta * Out(i, l),   i < s <= kThinMax, l < L,
// with X (k x L) at X[q*x_q + l*x_l], Y (s x k) at Y[i*y_i + q*y_q] and Out at O[i*o_i + l*o_l].
// A few rows of C: Y = those rows of op(A), X = op(B). A few columns: Y = op(B)^T restricted to
// them, X = op(A)^T. Each workgroup owns kThinL consecutive l and the whole k range: chunks of
// kThinKC k-values of X and Y are loaded with coalesced reads (along whichever of q or l has the
// unit stride), staged in LDS, and each thread accumulates 4 l's by S rows over one k-residue
// class mod 64; the 64 partial sums are then added in a fixed order (lanes, then waves), so the
// result does not depend on timing.
// ------------------------------------------------------------------------------------------------
struct ThinArgs {
  int64_t s, L, k;
  const double* X;
  int64_t x_q, x_l;
  const double* Y;
  int64_t y_i, y_q;
  double* O;
  int64_t o_i, o_l;
  double alpha, beta;
  int x_qfast, y_qfast;  // 1: the unit stride of X (of Y) runs along q; 0: along l (along i)
};

// Up to two thin blocks in one launch: workgroups [0, blocks0) take p[0], the rest p[1].
struct ThinPair {
  ThinArgs p[2];
  int blocks0;
};

constexpr int kThinMax = 16;          // largest thin side
constexpr int kThinL = 16;            // outputs along l per workgroup
constexpr int kThinKC = 256;          // k-values per staged chunk
constexpr int kThinXS = kThinL + 2;   // LDS row stride of the X chunk (rows stay 16-byte aligned)
constexpr int kThinYS = kThinKC + 2;  // LDS row stride of the Y chunk
// Largest leading dimension the thin kernel's 32-bit element offsets within a chunk allow.
constexpr int64_t kThinMaxLd = (int64_t)INT32_MAX / (kThinKC + kThinMax);

// The body for one layout of X (XQ: unit stride along q) and of Y (YQ: unit stride along q).
// Addresses are formed from a per-chunk base (uniform) plus a 32-bit element offset: the host
// only takes this path when (kThinKC-1)*|q stride| + (kThinL-1 or S-1)*|other stride| < 2^31.
// Two chunks are in flight: while one is multiplied out of LDS the next two are loading.
template <int S, bool XQ, bool YQ>
__device__ __forceinline__ void thin_body(const ThinArgs& a, int64_t l0, double* xs, double* ys) {
  const int t = threadIdx.x;
  // Element r of this thread's share of a chunk: X (16 per thread) and Y (S per thread). With
  // the unit stride along q a wave reads 64 consecutive q of one l (of one i); otherwise 4 rows
  // of 16 consecutive l (S consecutive i per q).
  const int xq0 = XQ ? t : (t >> 4), xl0 = XQ ? 0 : (t & 15);  // q = xq0 + xqs*r, l = xl0 + xls*r
  constexpr int xqs = XQ ? 0 : 16, xls = XQ ? 1 : 0;
  const int yi0 = YQ ? 0 : (t % S), yq0 = YQ ? t : t / S;
  constexpr int yis = YQ ? 1 : 0, yqs = YQ ? 0 : kThinKC / S;
  const int l_last = (int)min<int64_t>(a.L - 1 - l0, kThinL - 1);  // last valid l of this block
  const int i_last = (int)(a.s - 1);
  const int xq = (int)a.x_q, xl = (int)a.x_l, yi = (int)a.y_i, yq = (int)a.y_q;

  auto load_chunk = [&](int64_t q0, double (&xr)[16], double (&yr)[S]) {
    const int q_last = (int)min<int64_t>(a.k - 1 - q0, kThinKC - 1);
    const double* xb = a.X + q0 * a.x_q + l0 * a.x_l;
    const double* yb = a.Y + q0 * a.y_q;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int q = min(xq0 + xqs * r, q_last), l = min(xl0 + xls * r, l_last);
      xr[r] = xb[q * xq + l * xl];
    }
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const int i = min(yi0 + yis * r, i_last), q = min(yq0 + yqs * r, q_last);
      yr[r] = yb[i * yi + q * yq];
    }
  };
  // Values outside the operands (q >= k, l >= L, i >= s) go to LDS as zeros.
  auto store_chunk = [&](int64_t q0, const double (&xr)[16], const double (&yr)[S]) {
    const int64_t q_end = a.k - q0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int q = xq0 + xqs * r, l = xl0 + xls * r;
      xs[q * kThinXS + l] = (q < q_end && l <= l_last) ? xr[r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const int i = yi0 + yis * r, q = yq0 + yqs * r;
      ys[i * kThinYS + q] = (q < q_end && i <= i_last) ? yr[r] : 0.0;
    }
  };

  const int lq = t & 3, g = t >> 2;  // l = 4*lq .. 4*lq+3, k-residue g mod 64
  double acc[S][4];
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
  auto multiply = [&]() {
#pragma unroll
    for (int j = 0; j < kThinKC / 64; ++j) {
      const int q = g + 64 * j;
      const double2 x01 = *reinterpret_cast<const double2*>(&xs[q * kThinXS + 4 * lq]);
      const double2 x23 = *reinterpret_cast<const double2*>(&xs[q * kThinXS + 4 * lq + 2]);
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double y = ys[i * kThinYS + q];
        acc[i][0] = fma(y, x01.x, acc[i][0]);
        acc[i][1] = fma(y, x01.y, acc[i][1]);
        acc[i][2] = fma(y, x23.x, acc[i][2]);
        acc[i][3] = fma(y, x23.y, acc[i][3]);
      }
    }
  };

  const int64_t chunks = (a.k + kThinKC - 1) / kThinKC;
  double xa[16], ya[S], xb[16], yb[S];
  load_chunk(0, xa, ya);
  if (chunks > 1) load_chunk(kThinKC, xb, yb);
  for (int64_t c = 0; c < chunks; c += 2) {
    if (c > 0) __syncthreads();  // the previous chunk has been read
    store_chunk(c * kThinKC, xa, ya);
    __syncthreads();
    if (c + 2 < chunks) load_chunk((c + 2) * kThinKC, xa, ya);
    multiply();
    if (c + 1 >= chunks) break;
    __syncthreads();
    store_chunk((c + 1) * kThinKC, xb, yb);
    __syncthreads();
    if (c + 3 < chunks) load_chunk((c + 3) * kThinKC, xb, yb);
    multiply();
  }

  // The 16 residue classes of a wave (lane bits 2..5), then the 4 waves in order.
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int off = 4; off < 64; off <<= 1) acc[i][u] += __shfl_xor(acc[i][u], off);
  __syncthreads();  // xs is reused for the per-wave sums
  double* red = xs;  // [wave][i][l]
  const int wave = t >> 6;
  if ((t & 63) < 4) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) red[(wave * S + i) * kThinL + 4 * lq + u] = acc[i][u];
  }
  __syncthreads();
  if (t < S * kThinL) {
    const int i = t / kThinL, l = t % kThinL;
    if (i <= i_last && l <= l_last) {
      const double sum = ((red[i * kThinL + l] + red[(S + i) * kThinL + l]) +
                          red[(2 * S + i) * kThinL + l]) + red[(3 * S + i) * kThinL + l];
      double* o = a.O + i * a.o_i + (l0 + l) * a.o_l;
      const double v = a.alpha * sum;
      *o = (a.beta != 0.0) ? fma(a.beta, *o, v) : v;
    }
  }
}

template <int S>
__global__ void __launch_bounds__(256) thin_kernel(ThinPair tp) {
  static_assert(S == 4 || S == 8 || S == 16, "thin side bucket");
  __shared__ __align__(16) double xs[kThinKC * kThinXS];
  __shared__ double ys[S * kThinYS];
  const bool second = (int)blockIdx.x >= tp.blocks0;
  const ThinArgs& a = second ? tp.p[1] : tp.p[0];
  const int64_t l0 = (int64_t)(second ? (int)blockIdx.x - tp.blocks0 : (int)blockIdx.x) * kThinL;
  if (a.x_qfast) {
    if (a.y_qfast) thin_body<S, true, true>(a, l0, xs, ys);
    else           thin_body<S, true, false>(a, l0, xs, ys);
  } else {
    if (a.y_qfast) thin_body<S, false, true>(a, l0, xs, ys);
    else           thin_body<S, false, false>(a, l0, xs, ys);
  }
}

// ------------------------------------------------------------------------------------------------
// Wave tiles: one wave computes a 32 x 32 tile of C on its own, with no LDS and no barrier, so
// every wave of a workgroup (and of a CU) runs its own pipeline over its own list of tiles. This
// is the tile of the grouped launch's class 2 and of the single-GEMM "wave" variant.
//
// Fragments come straight from memory into registers, 16 bytes per lane per load, in k-steps of 8
// (two MFMA substeps). The MFMA k-index of lane group c (lanes 16c..16c+15) in substep e of step s
// is 8s + 2c + e, for both operands: the same k-sets in the same order as the ring kernels, so a
// wave tile returns the ring kernels' bits. The 32 rows of the tile are taken in pairs: lane l
// feeds rows 2(l%16) and 2(l%16) + 1 (MFMA blocks 0 and 1); the 32 columns likewise. A 16-byte
// load is then either one row pair (or column pair) at one k -- operands contiguous along m or n
// -- or a k-pair of one row (column) -- operands contiguous along k -- and four loads per wave
// cover a step. Lane l ends holding C(i0 + 2(l%16) + bi, j0 + 2(l/16 + 4r) + bj) in register r of
// block (bi, bj).
//
// Loads use buffer resources over the rest of each operand's storage (reads past its end give
// zero), per-lane 32-bit offsets within a step's panel and a scalar panel origin. Entries with
// k-index >= k are zero from the bound for operands contiguous along m or n; for operands
// contiguous along k they are zeroed in registers in the last step.
// ------------------------------------------------------------------------------------------------
typedef double d2 __attribute__((ext_vector_type(2)));
constexpr int kWT = 32;  // rows and columns of a wave tile
constexpr int kWK = 8;   // k per step

__device__ __forceinline__ d2 load_d2(rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
}

template <bool TA, bool TB>
__device__ __forceinline__ void wave_tile(const GemmArgs& g, int64_t i0, int64_t j0, int lane) {
  const int r16 = lane & 15, c = lane >> 4;
  // Per-lane byte offsets within a step's panel. TA: row 2 r16 + u, k-pair 2c; else k = 2c + u,
  // rows 2 r16 and 2 r16 + 1. TB: k = 2c + u, columns 2 r16, 2 r16 + 1; else column 2 r16 + u,
  // k-pair 2c.
  uint32_t offa[2], offb[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    offa[u] = (uint32_t)(8 * (TA ? (int64_t)(2 * r16 + u) * g.lda + 2 * c
                                 : (int64_t)(2 * c + u) * g.lda + 2 * r16));
    offb[u] = (uint32_t)(8 * (TB ? (int64_t)(2 * c + u) * g.ldb + 2 * r16
                                 : (int64_t)(2 * r16 + u) * g.ldb + 2 * c));
  }
  const int64_t a_org = TA ? i0 * g.lda : i0;
  const int64_t a_step = TA ? (int64_t)kWK : (int64_t)kWK * g.lda;
  const int64_t b_org = TB ? j0 : j0 * g.ldb;
  const int64_t b_step = TB ? (int64_t)kWK * g.ldb : (int64_t)kWK;

  d4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = (d4){0.0, 0.0, 0.0, 0.0};

  // alpha == 0 or k == 0: no product (A and B are not read); the epilogue forms beta*C.
  const int nsteps = (g.alpha == 0.0) ? 0 : (int)((g.k + kWK - 1) / kWK);
  const int k_last = (int)(g.k - (int64_t)(nsteps - 1) * kWK);  // k-values in the last step

  // Loads of step s.
  auto load = [&](int s, d2 (&xa)[2], d2 (&xb)[2]) {
    const int64_t ao = a_org + (int64_t)s * a_step, bo = b_org + (int64_t)s * b_step;
    const rsrc_t ra = make_rsrc(g.A + ao, g.ext_a - ao);
    const rsrc_t rb = make_rsrc(g.B + bo, g.ext_b - bo);
    xa[0] = load_d2(ra, offa[0]);
    xa[1] = load_d2(ra, offa[1]);
    xb[0] = load_d2(rb, offb[0]);
    xb[1] = load_d2(rb, offb[1]);
  };
  auto compute = [&](int s, d2 (&xa)[2], d2 (&xb)[2]) {
    if (s == nsteps - 1 && k_last < kWK) {  // uniform: zero k >= k in k-contiguous operands
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          if (TA && 2 * c + e >= k_last) xa[u][e] = 0.0;
          if (!TB && 2 * c + e >= k_last) xb[u][e] = 0.0;
        }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      double af[2], bf[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        af[b] = TA ? xa[b][e] : xa[e][b];
        bf[b] = TB ? xb[e][b] : xb[b][e];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[bj], af[bi], acc[bi][bj], 0, 0, 0);
    }
  };

  // Two steps of lookahead over a 3-deep register ring. The steady loop issues its loads
  // unconditionally (up to two steps past the end: through the buffer bound those read zeros or
  // other entries of the same storage, and are never used), so every path reaches each compute
  // with the same loads outstanding and the wait before it stays exact; the last one or two steps
  // drain without loads.
  d2 a0[2], b0[2], a1[2], b1[2], a2[2], b2[2];
  if (nsteps > 0) {
    load(0, a0, b0);
    load(1, a1, b1);
    int s = 0;
    for (; s + 3 <= nsteps; s += 3) {
      load(s + 2, a2, b2);
      compute(s, a0, b0);
      load(s + 3, a0, b0);
      compute(s + 1, a1, b1);
      load(s + 4, a1, b1);
      compute(s + 2, a2, b2);
    }
    if (s < nsteps) compute(s, a0, b0);
    if (s + 1 < nsteps) compute(s + 1, a1, b1);
  }

  // Epilogue: C(i,j) := alpha*acc + beta*C(i,j); with beta == 0 the old C is not read.
  const double alpha = g.alpha, beta = g.beta;
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = j0 + 2 * (c + 4 * r) + bj;
      if (j >= g.n) continue;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int64_t i = i0 + 2 * r16 + bi;
        if (i >= g.m) continue;
        double* cp = g.C + j * g.ldc + i;
        const double v = alpha * acc[bi][bj][r];
        *cp = (beta != 0.0) ? fma(beta, *cp, v) : v;
      }
    }
}

// Single-GEMM form: a workgroup of 4 waves covers a 64 x 64 tile of C as four independent wave
// tiles (wave w takes the 32 x 32 quarter (w % 2, w / 2)); tiles are dealt XCD-aware as for the
// other kernels.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
dgemm_wave_kernel(GemmArgs g, int tiles_m, int tiles_n) {
  int tm, tn;
  if (!tile_coords(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i0 = (int64_t)tm * 64 + kWT * (wave & 1), j0 = (int64_t)tn * 64 + kWT * (wave >> 1);
  if (i0 >= g.m || j0 >= g.n) return;
  wave_tile<TA, TB>(g, i0, j0, threadIdx.x & 63);
}

// ------------------------------------------------------------------------------------------------
// Ring kernels: the k-panels of op(A) and op(B) stream from memory straight into a ring of STAGES
// LDS stages (buffer loads with an LDS destination, no register staging), STAGES - 1 panels ahead
// of the arithmetic, and the MFMAs of each panel's last k-substeps are issued after the barrier
// that ends the panel, where they cover the LDS latency of the next panel's first fragments.
//
// A direct load moves 16 bytes per lane into LDS at (wave-uniform base) + 16 * lane, so a wave
// fills one 1 KB chunk per load. Each 16 bytes are two neighbours along the operand's stored
// (contiguous) dimension, which fixes two LDS layouts:
//   k-major (operand contiguous along m or n): a chunk is 128 consecutive rows of one k-row; k-rows
//     are R + 8 doubles apart, so that the fragment reads of k-rows two apart use disjoint halves
//     of the 64 LDS banks;
//   row-major (operand contiguous along k): each row holds the panel's 16 k-values as 8 pairs of
//     16 bytes, pair p of row i stored in slot p ^ f(i), f(i) = (i & 7) ^ ((i >> 3) & 1), which makes
//     16-byte fragment reads of 8 (32 banks) or 16 (64 banks) consecutive rows conflict-free.
// A fragment read of a k-pair serves two MFMAs, so the MFMA k-index of lane group c (lanes
// 16c..16c+15) in substep e of pair h is 8h + 2c + e; both operands use this order, which only
// permutes the terms of each panel's sum.
// ------------------------------------------------------------------------------------------------
template <int MT_, int NT_, int WM_, int WN_, int STAGES_, int MIN_WAVES_PER_EU_, int SCHED_ = 0,
          int KS_ = 1>
struct RingCfg {
  static constexpr int MT = MT_, NT = NT_, KT = 16, WM = WM_, WN = WN_, STAGES = STAGES_;
  // Instruction order inside a k-step. 0: each panel's fragment reads strictly before the MFMAs
  // they overlap; 1: MFMAs interleaved one by one with the direct loads and fragment reads, so
  // that the matrix pipe restarts at once after a barrier and LDS traffic is spread out.
  static constexpr int SCHED = SCHED_;
  // Wave groups splitting k inside the workgroup: group g multiplies the panels p with
  // p % KS == g of the tile's k-loop, each group an independent grid of WAVES_G waves with its
  // own part of every LDS stage, all groups in step at the same barriers. A stage then holds KS
  // panels, so each barrier covers KS panels of MFMA work and every SIMD runs KS waves. At the
  // end the groups add their partial tiles through LDS in a fixed order (the result does not
  // depend on timing) and each writes its share of C.
  static constexpr int KS = KS_;
  // Tile-rows per column group of the XCD-aware tile order: the 32 tiles resident on an XCD then
  // span GROUP tile-rows and 32 / GROUP tile-columns; 4 x 8 tiles of 256 x 128 touch the fewest
  // rows of op(A) plus columns of op(B) per k-panel (1024 + 1024).
  static constexpr int GROUP = MT > NT ? 4 : 8;
  static constexpr int MIN_WAVES_PER_EU = MIN_WAVES_PER_EU_;
  static constexpr int WAVES_M = MT / WM, WAVES_N = NT / WN;
  static constexpr int WAVES_G = WAVES_M * WAVES_N;  // waves per k-group
  static constexpr int WAVES = WAVES_G * KS;
  static constexpr int THREADS = WAVES * 64;
  static constexpr int BM = WM / 16, BN = WN / 16;
  static constexpr int PAIRS = KT / 8;  // k-pairs of MFMA substeps per panel
  // k-major row strides (doubles): 8 doubles of padding, except for 64-row tiles, whose 1 KB
  // direct loads fill two k-rows at once and use the XOR placement of kmaj_index instead.
  static constexpr int ROW_A = MT == 64 ? 64 : MT + 8, ROW_B = NT == 64 ? 64 : NT + 8;
  static constexpr int STAGE_A = KT * ROW_A, STAGE_B = KT * ROW_B;
  static constexpr int STAGE = STAGE_A + STAGE_B;  // one panel of one k-group
  static constexpr int SUPER = KS * STAGE;         // one ring slot: a panel per k-group
  static constexpr int LDS_DOUBLES = STAGES * SUPER;
  static constexpr int A_LOADS = MT * KT / 128 / WAVES_G, B_LOADS = NT * KT / 128 / WAVES_G;
  static constexpr int LOADS = A_LOADS + B_LOADS;  // direct loads per wave per panel
  static_assert((MT % 128 == 0 || MT == 64) && (NT % 128 == 0 || NT == 64),
                "k-major chunks are 128-row pieces of a k-row, or two k-rows of a 64-row tile");
  static_assert((MT * KT / 128) % WAVES_G == 0 && (NT * KT / 128) % WAVES_G == 0, "chunk split");
  static_assert(MT % WM == 0 && NT % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "wave grid");
  static_assert(STAGES >= 2 && STAGES <= 4 && (STAGES - 1) * LOADS <= 63, "vmcnt range");
  static_assert(THREADS <= 1024, "workgroup size");
  static_assert(KS == 1 || (KS == 2 && BN % 2 == 0 && MT * NT <= LDS_DOUBLES) ||
                    (KS == 4 && BM * BN == 4 && WAVES * 4 * 256 <= LDS_DOUBLES),
                "k-groups share the blocks of the epilogue through the LDS ring");
};

__device__ __forceinline__ int ring_swz(int row) { return (row & 7) ^ ((row >> 3) & 1); }

// LDS index (doubles, within an operand's stage) of element (k-row q, row i) of a k-major panel
// with ROWS rows and row stride ROW. For ROWS = 64 the rows are unpadded and k-rows whose index
// has bit 1 set are stored with bit 4 of the row index flipped (a 128-byte shift), so the
// fragment reads of k-rows two apart, issued by the two halves of a 32-lane phase, fall in
// opposite halves of the LDS banks.
template <int ROWS, int ROW>
__device__ __forceinline__ int kmaj_index(int q, int i) {
  if constexpr (ROWS == 64) return q * 64 + (i ^ (16 * ((q >> 1) & 1)));
  else return q * ROW + i;
}

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// Compiler-level ordering of LDS accesses around a bare s_barrier (which by itself does not keep
// the compiler from moving memory operations across it).
__device__ __forceinline__ void ring_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// s_waitcnt with vmcnt(N) and lgkmcnt(0), expcnt untouched (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N <= 63, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (0 << 8));
}

template <int LOADS, int MAXN>
__device__ __forceinline__ void wait_panels(int newer) {  // newer = panels allowed in flight
  if constexpr (MAXN >= 3) { if (newer >= 3) { wait_vm_lgkm0<3 * LOADS>(); return; } }
  if constexpr (MAXN >= 2) { if (newer == 2) { wait_vm_lgkm0<2 * LOADS>(); return; } }
  if constexpr (MAXN >= 1) { if (newer == 1) { wait_vm_lgkm0<1 * LOADS>(); return; } }
  wait_vm_lgkm0<0>();
}

// Scheduling-group patterns (sched_group_barrier masks: 0x008 MFMA, 0x020 VMEM read,
// 0x100 DS read): N times one MFMA followed by one instruction of class MASK.
template <int MASK, int N>
__device__ __forceinline__ void sched_mfma_then() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(MASK, 1, 0);
    sched_mfma_then<MASK, N - 1>();
  }
}

// N times: M MFMAs followed by one instruction of class MASK.
template <int M, int MASK, int N>
__device__ __forceinline__ void sched_mfmas_then() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x008, M, 0);
    __builtin_amdgcn_sched_group_barrier(MASK, 1, 0);
    sched_mfmas_then<M, MASK, N - 1>();
  }
}

// Per-lane global byte offset (from the panel origin) and wave-uniform LDS chunk base (doubles,
// within the operand's part of a stage) of direct load u of one operand with R panel rows.
template <class R, int ROWS, int ROW, bool CONTIG_K>
__device__ __forceinline__ void ring_map(int wave, int lane, int u, int64_t ld, uint32_t& off,
                                         int& lds) {
  const int c = wave + R::WAVES_G * u;
  if constexpr (!CONTIG_K && ROWS == 64) {
    // chunk c holds k-rows 2c (lanes 0-31) and 2c+1 (lanes 32-63); lane l writes doubles
    // 2(l & 31), +1 of its k-row, which kmaj_index assigns to rows i, i+1 below
    const int q = 2 * c + (lane >> 5);
    const int i = 2 * ((lane & 31) ^ (8 * ((q >> 1) & 1)));
    off = (uint32_t)((i + (int64_t)q * ld) * 8);
    lds = c * 128;
  } else if constexpr (!CONTIG_K) {
    constexpr int per_row = ROWS / 128;
    const int q = c / per_row, part = c % per_row;
    const int i = part * 128 + 2 * lane;
    off = (uint32_t)((i + (int64_t)q * ld) * 8);
    lds = q * ROW + part * 128;
  } else {
    const int i = c * 8 + (lane >> 3);
    const int p = (lane & 7) ^ ring_swz(i);
    off = (uint32_t)((2 * p + (int64_t)i * ld) * 8);
    lds = c * 128;
  }
}

// Zero the entries with k-index >= k_left of one panel (ragged last panel); the threads of one
// k-group (thread index gt of R::WAVES_G * 64) share the work.
template <class R, bool TA, bool TB>
__device__ __forceinline__ void ring_mask_tail(double* st, int k_left, int gt) {
  constexpr int kStride = R::WAVES_G * 64;
  double* As = st;
  double* Bs = st + R::STAGE_A;
  for (int e = gt; e < R::MT * R::KT; e += kStride) {
    if (!TA) {
      const int q = e / R::MT, i = e % R::MT;
      if (q >= k_left) As[kmaj_index<R::MT, R::ROW_A>(q, i)] = 0.0;
    }
    else { const int i = e / R::KT, q = e % R::KT;
           if (q >= k_left) As[i * R::KT + 2 * ((q >> 1) ^ ring_swz(i)) + (q & 1)] = 0.0; }
  }
  for (int e = gt; e < R::NT * R::KT; e += kStride) {
    if (TB) {
      const int q = e / R::NT, j = e % R::NT;
      if (q >= k_left) Bs[kmaj_index<R::NT, R::ROW_B>(q, j)] = 0.0;
    }
    else { const int j = e / R::KT, q = e % R::KT;
           if (q >= k_left) Bs[j * R::KT + 2 * ((q >> 1) ^ ring_swz(j)) + (q & 1)] = 0.0; }
  }
}

// Tile (tm, tn) of C by one workgroup of a ring configuration; `smem` holds R::LDS_DOUBLES.
// TRI restricts the epilogue to one triangle of C (0: all of it; 1: i >= j; 2: i <= j): entries
// outside it are neither read nor written.
template <class R, bool TA, bool TB, int TRI = 0>
__device__ __forceinline__ void ring_tile(const GemmArgs& g, int tm, int tn, double* smem) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave_all = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = R::KS == 1 ? 0 : wave_all / R::WAVES_G;  // k-group
  const int wave = R::KS == 1 ? wave_all : wave_all % R::WAVES_G;
  const int gtid = R::KS == 1 ? tid : tid - grp * R::WAVES_G * 64;
  const int wave_m = wave % R::WAVES_M, wave_n = wave / R::WAVES_M;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t row0 = (int64_t)tm * R::MT, col0 = (int64_t)tn * R::NT;

  // Direct-load placement (k-major for an operand contiguous along m or n).
  uint32_t a_off[R::A_LOADS], b_off[R::B_LOADS];
  int a_lds[R::A_LOADS], b_lds[R::B_LOADS];
#pragma unroll
  for (int u = 0; u < R::A_LOADS; ++u)
    ring_map<R, R::MT, R::ROW_A, TA>(wave, lane, u, g.lda, a_off[u], a_lds[u]);
#pragma unroll
  for (int u = 0; u < R::B_LOADS; ++u)
    ring_map<R, R::NT, R::ROW_B, !TB>(wave, lane, u, g.ldb, b_off[u], b_lds[u]);

  // Ring slot p holds k-panel KS * p + g of group g at offset g * STAGE; num_k counts slots.
  constexpr int KD = R::KS * R::KT;  // k-depth of one ring slot
  const int64_t a_gk = TA ? (int64_t)R::KT : (int64_t)R::KT * g.lda;  // one panel along k
  const int64_t b_gk = TB ? (int64_t)R::KT * g.ldb : (int64_t)R::KT;
  const int64_t a_org = (TA ? row0 * g.lda : row0) + grp * a_gk;
  const int64_t a_step = R::KS * a_gk;
  const int64_t b_org = (TB ? col0 : col0 * g.ldb) + grp * b_gk;
  const int64_t b_step = R::KS * b_gk;
  double* const gsm = smem + grp * R::STAGE;  // this group's part of slot 0

  const int num_k = (g.alpha == 0.0) ? 0 : (int)((g.k + KD - 1) / KD);
  const int k_left_last = (int)(g.k - (int64_t)(num_k - 1) * KD);  // 1..KD
  // k-entries of this group's panel in the last slot: KT, fewer, or none (then the whole panel
  // is masked; its loads start past the operand's end or are masked like any k-tail)
  const int k_left_grp =
      R::KS == 1 ? k_left_last : min(max(k_left_last - grp * R::KT, 0), R::KT);

  auto issue = [&](int p) {
    double* st = gsm + (p % R::STAGES) * R::SUPER;
    const int64_t ao = a_org + p * a_step, bo = b_org + p * b_step;
    const rsrc_t ra = make_rsrc(g.A + ao, g.ext_a - ao);
    const rsrc_t rb = make_rsrc(g.B + bo, g.ext_b - bo);
#pragma unroll
    for (int u = 0; u < R::A_LOADS; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void_ptr)(st + a_lds[u]), 16, a_off[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < R::B_LOADS; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_ptr)(st + R::STAGE_A + b_lds[u]), 16,
                                               b_off[u], 0, 0, 0);
  };

  // Fragment addresses (doubles from the stage base) of this lane for pair 0; pair h adds h * 8
  // k-rows (k-major) or flips slot bit 2 (row-major: slot (4h + c) ^ f = (4h) ^ (c ^ f)).
  // Row-major: lane l16 feeds row ai + 16b of block b, and one 16-byte read gives it the k-values
  // of both k-steps e of the pair.
  // k-major: one 16-byte read gives lane l16 rows 2*l16 and 2*l16 + 1 of a 32-row group at one
  // k-row (2*lq + 8h + e), which feed k-step e of two MFMA blocks: block 2p holds the group's even
  // rows, block 2p + 1 its odd rows (the epilogue maps them back). In a 64-row tile, k-rows
  // 2*lq + 8h + e all have bit 1 equal to lq & 1, so kmaj_index flips bit 4 of the row for odd lq
  // (the wave's rows start at a multiple of 32): the pair moves to (2*l16) ^ 16.
  const int ai = wave_m * R::WM + l16, bj = wave_n * R::WN + l16;
  const int kflip = lq & 1;
  static_assert(R::MT != 64 || R::WM % 32 == 0, "64-row tiles: wave rows start at multiples of 32");
  static_assert(R::NT != 64 || R::WN % 32 == 0, "64-row tiles: wave rows start at multiples of 32");
  static_assert(R::BM % 2 == 0 && R::BN % 2 == 0, "k-major reads feed blocks in pairs");
  const int a_rmaj = ai * R::KT + 2 * (lq ^ ring_swz(l16));
  const int b_rmaj = R::STAGE_A + bj * R::KT + 2 * (lq ^ ring_swz(l16));
  const int a_kp = 2 * lq * R::ROW_A + wave_m * R::WM +
                   (R::MT == 64 ? ((2 * l16) ^ (16 * kflip)) : 2 * l16);
  const int b_kp = R::STAGE_A + 2 * lq * R::ROW_B + wave_n * R::WN +
                   (R::NT == 64 ? ((2 * l16) ^ (16 * kflip)) : 2 * l16);

  typedef double d2 __attribute__((ext_vector_type(2)));
  auto read_frags = [&](const double* st, int h, d2 (&fa)[R::BM], d2 (&fb)[R::BN]) {
    if constexpr (!TA) {
#pragma unroll
      for (int p = 0; p < R::BM / 2; ++p) {
        const double* q = st + a_kp + 8 * h * R::ROW_A + 32 * p;
        const d2 t0 = *reinterpret_cast<const d2*>(q);
        const d2 t1 = *reinterpret_cast<const d2*>(q + R::ROW_A);
        fa[2 * p] = (d2){t0[0], t1[0]};
        fa[2 * p + 1] = (d2){t0[1], t1[1]};
      }
    } else {
#pragma unroll
      for (int b = 0; b < R::BM; ++b)
        fa[b] = *reinterpret_cast<const d2*>(st + ((a_rmaj + 16 * b * R::KT) ^ (8 * h)));
    }
    if constexpr (TB) {
#pragma unroll
      for (int p = 0; p < R::BN / 2; ++p) {
        const double* q = st + b_kp + 8 * h * R::ROW_B + 32 * p;
        const d2 t0 = *reinterpret_cast<const d2*>(q);
        const d2 t1 = *reinterpret_cast<const d2*>(q + R::ROW_B);
        fb[2 * p] = (d2){t0[0], t1[0]};
        fb[2 * p + 1] = (d2){t0[1], t1[1]};
      }
    } else {
#pragma unroll
      for (int b = 0; b < R::BN; ++b)
        fb[b] = *reinterpret_cast<const d2*>(st + ((b_rmaj + 16 * b * R::KT) ^ (8 * h)));
    }
  };

  d4 acc[R::BM][R::BN];
#pragma unroll
  for (int i = 0; i < R::BM; ++i)
#pragma unroll
    for (int j = 0; j < R::BN; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  auto mfma_pair = [&](const d2 (&fa)[R::BM], const d2 (&fb)[R::BN]) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int i = 0; i < R::BM; ++i)
#pragma unroll
        for (int j = 0; j < R::BN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j][e], fa[i][e], acc[i][j], 0, 0, 0);
  };

  if (num_k > 0) {
    // Panels 0 .. STAGES-1 fill the ring; panel p + STAGES goes into p's slot right after the
    // barrier that ends panel p, so loads run about STAGES - 1 panels ahead of their use.
    const int pre = num_k < R::STAGES ? num_k : R::STAGES;
    for (int p = 0; p < pre; ++p) issue(p);
    wait_panels<R::LOADS, R::STAGES - 1>(pre - 1);
    ring_barrier();
    if (num_k == 1 && k_left_last < KD) {
      ring_mask_tail<R, TA, TB>(gsm, k_left_grp, gtid);
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
      ring_barrier();
    }
    d2 fa0[R::BM], fb0[R::BN], fa1[R::BM], fb1[R::BN];
    read_frags(gsm, 0, fa0, fb0);
    // 16-byte fragment reads per read_frags: one per block (row-major), two per pair of blocks
    // (k-major).
    constexpr int kReads = R::BM + R::BN;
    int t = 0;
    // Steady state: every iteration issues a full panel of loads and the panel read after its
    // barrier is not the last one (which may need its k-tail masked), so the body has a single
    // path. Pair 1 of panel t is multiplied after the barrier that ends the panel.
    for (; t + R::STAGES < num_k && t + 2 < num_k; ++t) {
      const double* st = gsm + (t % R::STAGES) * R::SUPER;
      read_frags(st, 1, fa1, fb1);
      if (R::SCHED == 0) __builtin_amdgcn_sched_barrier(0);  // reads ahead of the MFMAs below
      mfma_pair(fa0, fb0);
      if (R::SCHED == 1) sched_mfma_then<0x100, kReads>();
      wait_vm_lgkm0<(R::STAGES - 2) * R::LOADS>();
      ring_barrier();
      issue(t + R::STAGES);
      read_frags(gsm + ((t + 1) % R::STAGES) * R::SUPER, 0, fa0, fb0);
      if (R::SCHED == 0) __builtin_amdgcn_sched_barrier(0);
      mfma_pair(fa1, fb1);
      if (R::SCHED == 1) {
        sched_mfma_then<0x100, kReads>();
        sched_mfmas_then<2, 0x020, R::LOADS>();
      }
    }
    // Drain: the last panels are loaded or in flight; the last one may need its k-tail masked.
    for (; t < num_k - 1; ++t) {
      const double* st = gsm + (t % R::STAGES) * R::SUPER;
      read_frags(st, 1, fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pair(fa0, fb0);
      const int last_issued = (t + R::STAGES - 1 < num_k) ? t + R::STAGES - 1 : num_k - 1;
      wait_panels<R::LOADS, R::STAGES - 2>(last_issued - (t + 1));
      ring_barrier();
      if (t + R::STAGES < num_k) issue(t + R::STAGES);
      const double* nst = gsm + ((t + 1) % R::STAGES) * R::SUPER;
      if (t + 1 == num_k - 1 && k_left_last < KD) {
        ring_mask_tail<R, TA, TB>(const_cast<double*>(nst), k_left_grp, gtid);
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        ring_barrier();
      }
      read_frags(nst, 0, fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      mfma_pair(fa1, fb1);
    }
    read_frags(gsm + ((num_k - 1) % R::STAGES) * R::SUPER, 1, fa1, fb1);
    mfma_pair(fa0, fb0);
    mfma_pair(fa1, fb1);
  }

  // Two k-groups: group g keeps column blocks [g BN/2, (g+1) BN/2) of its wave's tile and hands
  // the others to the group that keeps them, through the (drained) LDS ring. Each entry becomes
  // (group 0's sum) + (group 1's sum), the same value whichever group adds it.
  constexpr int kHalf = R::KS == 4 ? 1 : R::BN / R::KS;  // (four groups return before its use)
  if constexpr (R::KS == 2) {
    constexpr int kPer = R::BM * kHalf * 4 * 64;  // doubles one wave hands over
    ring_barrier();  // every wave is past its last fragment read; no direct load is in flight
    double* mine = smem + (grp * R::WAVES_G + wave) * kPer;
    const double* theirs = smem + ((1 - grp) * R::WAVES_G + wave) * kPer;
#pragma unroll
    for (int bj = 0; bj < R::BN; ++bj) {
      if (bj / kHalf == grp) continue;
#pragma unroll
      for (int bi = 0; bi < R::BM; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          mine[((bi * kHalf + bj % kHalf) * 4 + r) * 64 + lane] = acc[bi][bj][r];
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    ring_barrier();
#pragma unroll
    for (int bj = 0; bj < R::BN; ++bj) {
      if (bj / kHalf != grp) continue;
#pragma unroll
      for (int bi = 0; bi < R::BM; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[bi][bj][r] += theirs[((bi * kHalf + bj % kHalf) * 4 + r) * 64 + lane];
    }
  }

  // Epilogue: C(i,j) := alpha*acc + beta*C(i,j), rounded as fma(beta, C, alpha*acc) on every
  // path; with beta == 0 the old C is not read. Block bi
  // holds rows 16*bi + l16 of the wave's rows (row-major op(A)) or, read in row pairs, rows
  // 32*(bi/2) + 2*l16 + bi%2 (k-major op(A)); columns likewise with lq + 4r in place of l16.
  const double alpha = g.alpha, beta = g.beta;
  auto row_of = [&](int bi) -> int64_t {
    return row0 + wave_m * R::WM + (TA ? 16 * bi + l16 : 32 * (bi >> 1) + 2 * l16 + (bi & 1));
  };
  auto col_of = [&](int bj2, int r) -> int64_t {
    return col0 + wave_n * R::WN +
           (TB ? 32 * (bj2 >> 1) + 2 * (lq + 4 * r) + (bj2 & 1) : 16 * bj2 + lq + 4 * r);
  };

  // Four k-groups: every wave hands all four of its blocks to the LDS ring; group g then owns
  // block (g / BN, g % BN) of its wave's tile, adds the four groups' partial sums in group order
  // (the same value whichever group adds it) and writes that block of C.
  if constexpr (R::KS == 4) {
    ring_barrier();  // every wave is past its last fragment read; no direct load is in flight
    double* mine = smem + (grp * R::WAVES_G + wave) * 4 * 256;
#pragma unroll
    for (int bi = 0; bi < R::BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < R::BN; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[((bi * R::BN + bj) * 4 + r) * 64 + lane] = acc[bi][bj][r];
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    ring_barrier();
    const int bi_o = grp / R::BN, bj_o = grp % R::BN;
    double sum[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = ((grp * 4 + r) * 64) + lane;  // block grp of each group's wave slot
      sum[r] = ((smem[(0 * R::WAVES_G + wave) * 1024 + e] + smem[(1 * R::WAVES_G + wave) * 1024 + e]) +
                smem[(2 * R::WAVES_G + wave) * 1024 + e]) + smem[(3 * R::WAVES_G + wave) * 1024 + e];
    }
    const int64_t i = row_of(bi_o);
    double cb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = col_of(bj_o, r);
      cb[r] = (beta != 0.0 && i < g.m && j < g.n) ? g.C[j * g.ldc + i] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = col_of(bj_o, r);
      if (i < g.m && j < g.n) {
        const double v = alpha * sum[r];
        g.C[j * g.ldc + i] = (beta != 0.0) ? fma(beta, cb[r], v) : v;
      }
    }
    return;
  }
  // A tile wholly inside C (outside the triangle masking) takes a path with no condition on any
  // load or store: under per-element conditions the compiler cannot count the memory operations
  // in flight and waits for each store to complete before the next one goes out.
  if (TRI == 0 && row0 + R::MT <= g.m && col0 + R::NT <= g.n) {
#pragma unroll
    for (int bj2 = 0; bj2 < R::BN; ++bj2) {
      if (bj2 / kHalf != grp) continue;
      if (beta != 0.0) {
        double cb[R::BM][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int bi = 0; bi < R::BM; ++bi) cb[bi][r] = g.C[col_of(bj2, r) * g.ldc + row_of(bi)];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int bi = 0; bi < R::BM; ++bi)
            g.C[col_of(bj2, r) * g.ldc + row_of(bi)] = fma(beta, cb[bi][r], alpha * acc[bi][bj2][r]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int bi = 0; bi < R::BM; ++bi)
            g.C[col_of(bj2, r) * g.ldc + row_of(bi)] = alpha * acc[bi][bj2][r];
      }
    }
    return;
  }
#pragma unroll
  for (int bj2 = 0; bj2 < R::BN; ++bj2) {
    if (bj2 / kHalf != grp) continue;
    double cb[R::BM][4];
    if (beta != 0.0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = col_of(bj2, r);
        const bool col_ok = j < g.n;
#pragma unroll
        for (int bi = 0; bi < R::BM; ++bi) {
          const int64_t i = row_of(bi);
          const bool tri_ok = TRI == 0 || (TRI == 1 ? i >= j : i <= j);
          cb[bi][r] = (col_ok && i < g.m && tri_ok) ? g.C[j * g.ldc + i] : 0.0;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = col_of(bj2, r);
      if (j >= g.n) continue;
#pragma unroll
      for (int bi = 0; bi < R::BM; ++bi) {
        const int64_t i = row_of(bi);
        const bool tri_ok = TRI == 0 || (TRI == 1 ? i >= j : i <= j);
        if (i < g.m && tri_ok) {
          const double v = alpha * acc[bi][bj2][r];
          g.C[j * g.ldc + i] = (beta != 0.0) ? fma(beta, cb[bi][r], v) : v;
        }
      }
    }
  }
}

template <class R, bool TA, bool TB>
__global__ void __launch_bounds__(R::THREADS) __attribute__((amdgpu_waves_per_eu(R::MIN_WAVES_PER_EU)))
dgemm_ring_kernel(GemmArgs g, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(16))) double smem[R::LDS_DOUBLES];
  int tm, tn;
  if (!tile_coords<R::GROUP>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn)) return;
  ring_tile<R, TA, TB>(g, tm, tn, smem);
}

// ------------------------------------------------------------------------------------------------
// Symmetric rank-k update C := alpha*op(A)*op(A)^T + beta*C on one triangle of C: the GEMM with
// B = A (transb the opposite of trans) over the tiles that meet the triangle, each computed by
// the ring tile with its epilogue masked to the triangle.
//
// C is cut into square super-tiles of side S = SR * MT = SC * NT (SR x SC tiles each). The
// super-tiles on and below the diagonal (for the upper triangle: on and above) are numbered
// u = 0, 1, ... line by line, line a holding a + 1 of them, so that u < a (a+1)/2 + (a+1) within
// line a; workgroup t takes tile t % (SR SC) of super-tile t / (SR SC), going down the tile
// columns. Workgroups on one XCD take consecutive t (as in tile_coords) and so work on one or two
// super-tiles at a time, which share their SR row panels and SC column panels. Tiles beyond the
// edge of C or wholly outside the triangle (in the diagonal super-tiles) exit at once.
// ------------------------------------------------------------------------------------------------
template <class R>
struct SyrkGeom {
  static constexpr int S = 4 * (R::MT > R::NT ? R::MT : R::NT);  // super-tile side
  static constexpr int SR = S / R::MT, SC = S / R::NT;          // tiles per super-tile side
  static_assert(S % R::MT == 0 && S % R::NT == 0, "square super-tiles");
};

__device__ __forceinline__ void tri_decode(int u, int& a, int& b) {
  int x = (int)((sqrt(1.0 + 8.0 * (double)u) - 1.0) * 0.5);
  while ((int64_t)(x + 1) * (x + 2) / 2 <= u) ++x;  // correct a rounding of the root
  while (x > 0 && (int64_t)x * (x + 1) / 2 > u) --x;
  a = x;
  b = u - x * (x + 1) / 2;
}

template <class R, bool TA, bool TB, int TRI>
__global__ void __launch_bounds__(R::THREADS) __attribute__((amdgpu_waves_per_eu(R::MIN_WAVES_PER_EU)))
dsyrk_ring_kernel(GemmArgs g, int wgs, int64_t leaf) {
  static_assert(TRI == 1 || TRI == 2, "one triangle");
  using G = SyrkGeom<R>;
  __shared__ __attribute__((aligned(16))) double smem[R::LDS_DOUBLES];
  // Diagonal block blockIdx.y of C, of order `leaf` (the last one may be smaller; one block of
  // order n when the launch covers all of C): its rows and columns, and the rows of op(A) and
  // columns of op(B) it needs, start at blockIdx.y * leaf.
  const int64_t o = (int64_t)blockIdx.y * leaf;
  const int64_t ao = TA ? o * g.lda : o;
  GemmArgs gb = g;
  gb.m = gb.n = min(leaf, g.n - o);
  gb.A = g.A + ao;
  gb.B = g.B + ao;
  gb.C = g.C + o * (g.ldc + 1);
  gb.ext_a = g.ext_a - ao;
  gb.ext_b = g.ext_b - ao;
  // Contiguous ranges of t per XCD, as in tile_coords (the grid is a multiple of kXcds).
  const int t = (blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
  if (t >= wgs) return;
  int a, b;
  tri_decode(t / (G::SR * G::SC), a, b);  // super-tile on line a, b-th on it (b <= a)
  const int r = t % (G::SR * G::SC);
  const int srow = TRI == 1 ? a : b, scol = TRI == 1 ? b : a;
  const int tm = srow * G::SR + r % G::SR, tn = scol * G::SC + r / G::SR;
  const int64_t r0 = (int64_t)tm * R::MT, r1 = r0 + R::MT - 1;  // rows of the tile
  const int64_t c0 = (int64_t)tn * R::NT, c1 = c0 + R::NT - 1;  // columns of the tile
  if (r0 >= gb.m || c0 >= gb.n) return;          // beyond the edge of the block
  if (TRI == 1 ? r1 < c0 : r0 > c1) return;      // wholly outside the triangle
  ring_tile<R, TA, TB, TRI>(gb, tm, tn, smem);
}

// C := beta*C on one triangle of the n x n C (lower: i >= j, else i <= j); beta == 0 writes zeros
// without reading C. The whole update when alpha == 0 or k == 0.
__global__ void __launch_bounds__(256) scale_tri_kernel(int64_t n, int lower, double beta,
                                                        double* C, int64_t ldc) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / n, i = e - j * n;
    if (lower ? i < j : i > j) continue;
    double* c = C + j * ldc + i;
    *c = (beta == 0.0) ? 0.0 : beta * *c;
  }
}

// ------------------------------------------------------------------------------------------------
// Variant table.
// ------------------------------------------------------------------------------------------------
using Small = Cfg<64, 64, 16, 32, 32, 4, 0>;     // 4 waves, each 32x32 (4 MFMA chains)
using Mid8 = Cfg<128, 64, 16, 32, 32, 6, 0>;     // 8 waves, each 32x32
using Tiny = Cfg<32, 32, 16, 16, 16, 8, 0>;      // 4 waves, each 16x16 (one MFMA chain)
using Ring256i = RingCfg<256, 128, 64, 32, 3, 4, 1>;    // 16 waves of 64x32, 3 stages, interleaved
using Ring128x4i = RingCfg<128, 128, 32, 32, 4, 4, 1>;  // 16 waves of 32x32, 4 stages, interleaved
using Ring256wi = RingCfg<256, 128, 64, 64, 3, 2, 1>;   // 8 waves of 64x64, interleaved issue
using Ring64s3 = RingCfg<64, 64, 32, 32, 3, 3, 1>;      // 4 waves of 32x32, 3 stages, 3 WGs per CU
using Ring64s4 = RingCfg<64, 64, 32, 32, 4, 2, 1>;      // 4 stages, 2 WGs per CU
using Ring128x64 = RingCfg<128, 64, 32, 32, 3, 4, 1>;   // 8 waves of 32x32, 3 stages, 2 WGs per CU
using Ring128x256wi = RingCfg<128, 256, 64, 64, 3, 2, 1>;  // 8 waves of 64x64 on a wide tile, 3 stages
using Ring256x128t = RingCfg<256, 128, 128, 32, 3, 2, 1>;  // 8 waves of 128x32, 3 stages
using Ring128x256t = RingCfg<128, 256, 128, 32, 3, 2, 1>;  // 8 waves of 128x32 on a wide tile
// Two k-groups of 4 waves of 32x32 on a 64x64 tile, 4 stages: two waves per SIMD with one
// workgroup per CU.
using Ring64k2 = RingCfg<64, 64, 32, 32, 4, 2, 1, 2>;
// Two k-groups of 4 waves of 64x64 on a 128x128 tile, 2 stages (139 KB of LDS).
using Ring128k2 = RingCfg<128, 128, 64, 64, 2, 2, 1, 2>;
// Four k-groups of 4 waves of 32x32 on a 64x64 tile, 2 ring slots of four panels (128 KB of LDS).
using Ring64k4 = RingCfg<64, 64, 32, 32, 2, 4, 1, 4>;

typedef void (*KernelFn)(GemmArgs, int, int);

constexpr int kLdsPerCU = 160 * 1024;  // bytes of LDS per CU on gfx950

struct Variant {
  const char* name;
  int mt, nt, kt, threads;
  int wgs_per_cu;   // workgroups resident per CU (LDS- and register-limited)
  int eff_permil[2][2];  // [transa][transb]: measured share of the FP64 MFMA peak on large
                         // square shapes, per mille; 0 keeps the variant out of the automatic
                         // choice. For a two-group variant: the share measured on grids of at
                         // most one tile per CU, the only grids it is priced on
  int short_k_permil;    // the same share measured on m = n = 8192, k = 64 (HBM-bound: the old
                         // C streams in and out); 0 keeps the variant out of the choice for
                         // k <= kShortK
  KernelFn fn[2][2];  // [transa][transb]
  int ks;             // k-groups per workgroup (ring configurations; 1 elsewhere)
};

template <class C>
constexpr int resident_wgs() {
  // LDS footprint with the larger (padded) row stride of either operand layout.
  constexpr int lds = 2 * C::KT * 8 * (LdsLayout<C, false, true>::A + LdsLayout<C, true, false>::B);
  constexpr int by_lds = kLdsPerCU / lds;
  constexpr int by_waves = (C::MIN_WAVES_PER_EU * 4) / C::WAVES;
  return by_lds < by_waves ? by_lds : by_waves;
}

struct Eff {
  int nn, nt, tn, tt;
  constexpr Eff(int all) : nn(all), nt(all), tn(all), tt(all) {}
  constexpr Eff(int nn_, int nt_, int tn_, int tt_) : nn(nn_), nt(nt_), tn(tn_), tt(tt_) {}
};

template <class R>
constexpr Variant make_ring_variant(const char* name, Eff e, int short_k = 0) {
  constexpr int by_lds = kLdsPerCU / (R::LDS_DOUBLES * 8);
  constexpr int by_waves = (R::MIN_WAVES_PER_EU * 4) / R::WAVES;
  constexpr int wgs = by_lds < by_waves ? by_lds : by_waves;
  return Variant{name, R::MT, R::NT, R::KT, R::THREADS, wgs > 0 ? wgs : 1,
                 {{e.nn, e.nt}, {e.tn, e.tt}}, short_k,
                 {{dgemm_ring_kernel<R, false, false>, dgemm_ring_kernel<R, false, true>},
                  {dgemm_ring_kernel<R, true, false>, dgemm_ring_kernel<R, true, true>}},
                 R::KS};
}

template <class C>
constexpr Variant make_variant(const char* name, Eff e, int short_k = 0) {
  return Variant{name,
                 C::MT,
                 C::NT,
                 C::KT,
                 C::THREADS,
                 resident_wgs<C>() > 0 ? resident_wgs<C>() : 1,
                 {{e.nn, e.nt}, {e.tn, e.tt}}, short_k,
                 {{dgemm_mfma_kernel<C, false, false>, dgemm_mfma_kernel<C, false, true>},
                  {dgemm_mfma_kernel<C, true, false>, dgemm_mfma_kernel<C, true, true>}},
                 1};
}

// The single-GEMM form of the wave tiles: 64x64 per workgroup as four independent 32x32 wave
// tiles, no LDS; 4 workgroups per CU (register-limited).
constexpr Variant make_wave_variant(const char* name, Eff e, int short_k = 0) {
  return Variant{name, 64, 64, kWK, 256, 4, {{e.nn, e.nt}, {e.tn, e.tt}}, short_k,
                 {{dgemm_wave_kernel<false, false>, dgemm_wave_kernel<false, true>},
                  {dgemm_wave_kernel<true, false>, dgemm_wave_kernel<true, true>}},
                 1};
}

// Efficiencies are the measured TFLOP/s of each variant at m = n = k = 8192..16384 divided by
// 78.6 (per transpose case where given as four numbers, NN NT TN TT).
const Variant kVariants[] = {
    make_variant<Small>("mfma_f64_64x64x16_w32x32", 760, 360),
    make_variant<Mid8>("mfma_f64_128x64x16_w32x32", 790, 446),
    make_variant<Tiny>("mfma_f64_32x32x16_w16x16", 0),
    make_ring_variant<Ring256i>("ring_f64_256x128x16_w64x32_s3_il", Eff(932, 941, 927, 925)),
    make_ring_variant<Ring128x4i>("ring_f64_128x128x16_w32x32_s4_il", Eff(889, 902, 896, 896)),
    make_ring_variant<Ring256wi>("ring_f64_256x128x16_w64x64_s3_il", Eff(915, 940, 940, 948)),
    make_ring_variant<Ring64s3>("ring_f64_64x64x16_w32x32_s3_il", Eff(827, 855, 836, 834), 393),
    make_ring_variant<Ring64s4>("ring_f64_64x64x16_w32x32_s4_il", Eff(804, 821, 827, 797)),
    make_ring_variant<Ring128x64>("ring_f64_128x64x16_w32x32_s3_il", Eff(875, 905, 891, 875), 400),
    make_ring_variant<Ring128x256wi>("ring_f64_128x256x16_w64x64_s3_il", Eff(936, 947, 940, 946)),
    make_ring_variant<Ring256x128t>("ring_f64_256x128x16_w128x32_s3_il", Eff(935, 939, 946, 945)),
    make_ring_variant<Ring128x256t>("ring_f64_128x256x16_w128x32_s3_il", Eff(947, 938, 936, 946)),
    make_wave_variant("wave_f64_64x64x8_w32x32", 0),
    make_ring_variant<Ring64k2>("ringk2_f64_64x64x16_w32x32_s4", 0),
    // one round of 128x128 tiles: 2048^3 at 63.7-70.5 and 2048^2 x 8192 at 72.5-73.7 TFLOP/s, 3-5%
    // above the one-group 128x128 and 128x64 tiles
    make_ring_variant<Ring128k2>("ringk2_f64_128x128x16_w64x64_s2", Eff(946, 946, 946, 946)),
    make_ring_variant<Ring64k4>("ringk4_f64_64x64x16_w32x32_s2", 0),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Ring configurations that run the symmetric rank-k update. Each is named by the GEMM variant
// with the same configuration, whose tile shape, residency and measured efficiencies the choice
// uses; each runs either triangle.
typedef void (*SyrkFn)(GemmArgs, int, int64_t);

struct SyrkVariant {
  const char* name;  // the variant of kVariants with this ring configuration
  int super_side;    // side of the square super-tiles, in elements
  SyrkFn fn[2][2];   // [trans][upper]: trans 'N' runs the GEMM case NT, 'T' the case TN
};

template <class R>
constexpr SyrkVariant make_syrk_variant(const char* name) {
  return SyrkVariant{name, SyrkGeom<R>::S,
                     {{dsyrk_ring_kernel<R, false, true, 1>, dsyrk_ring_kernel<R, false, true, 2>},
                      {dsyrk_ring_kernel<R, true, false, 1>, dsyrk_ring_kernel<R, true, false, 2>}}};
}

const SyrkVariant kSyrkVariants[] = {
    make_syrk_variant<Ring256x128t>("ring_f64_256x128x16_w128x32_s3_il"),
    make_syrk_variant<Ring128x256wi>("ring_f64_128x256x16_w64x64_s3_il"),
    make_syrk_variant<Ring128x64>("ring_f64_128x64x16_w32x32_s3_il"),
    make_syrk_variant<Ring128x4i>("ring_f64_128x128x16_w32x32_s4_il"),
    make_syrk_variant<Ring64s3>("ring_f64_64x64x16_w32x32_s3_il"),
};
constexpr int kNumSyrkVariants = sizeof(kSyrkVariants) / sizeof(kSyrkVariants[0]);

// ------------------------------------------------------------------------------------------------
// Grouped launch: many independent GEMMs in one persistent kernel.
//
// A plan (built on the host, copied to the device by the caller) holds one descriptor per GEMM and
// a list of tiles (gemm, tm, tn) in schedule order. There are two kinds of plan.
//  - Workgroup tiles (classes 0 and 1): workgroup w processes list entries w, w + G, w + 2G, ...
//    (G = grid size) with the same tile code the single-GEMM kernels use: class 0 is the 64x64
//    tile of variant "mfma_f64_64x64x16_w32x32", class 1 the 32x32 tile of
//    "mfma_f64_32x32x16_w16x16".
//  - Wave tiles (class 2, every GEMM of the plan): each wave computes 32x32 tiles on its own
//    (wave_tile, as variant "wave_f64_64x64x8_w32x32"). The host gives every GEMM to one XCD (the
//    longest first, each to the XCD with the least work so far) and lists each XCD's tiles GEMM by
//    GEMM; the waves of the workgroups on XCD x walk x's list with a stride of their number, so the
//    waves working on one GEMM share its panels in that XCD's L2.
// Nothing is allocated or cleared at launch time, so a launch can be captured in a graph and
// replayed.
// ------------------------------------------------------------------------------------------------
using GroupedCfg0 = Small;
using GroupedCfg1 = Tiny;
constexpr int kGroupedClasses = 3;
constexpr int kWaveClass = 2;
constexpr int kGroupedThreads = 256;
static_assert(GroupedCfg0::THREADS == kGroupedThreads && GroupedCfg1::THREADS == kGroupedThreads,
              "grouped tile classes share one workgroup size");
constexpr int kPlanMagic = 0x4D444750;  // "MDGP"

struct GroupedDesc {
  GemmArgs g;
  int32_t ta, tb, tile_class, tiles_m;
  int32_t tiles_n, pad0, pad1, pad2;
};

struct PlanHeader {
  int32_t magic, version, count, kind;  // kind: 0 workgroup tiles, 1 wave tiles
  int64_t num_tiles;
  int64_t desc_offset, tile_offset;  // bytes from the plan start
  int64_t pad2[3];
};
static_assert(sizeof(PlanHeader) == 64, "plan header layout");
// A wave-tile plan has, right after the header, the tile-list offsets of the 8 XCDs' sublists
// (int64 [kXcds + 1], entries of the tile list), padded to kXcdTableBytes.
constexpr int kXcdTableBytes = 80;

constexpr int ilog_max(int a, int b) { return a > b ? a : b; }
constexpr int kGroupedLds = ilog_max(
    ilog_max(ilog_max(tile_lds_doubles<GroupedCfg0, false, false>(), tile_lds_doubles<GroupedCfg0, true, true>()),
             ilog_max(tile_lds_doubles<GroupedCfg0, false, true>(), tile_lds_doubles<GroupedCfg0, true, false>())),
    ilog_max(ilog_max(tile_lds_doubles<GroupedCfg1, false, false>(), tile_lds_doubles<GroupedCfg1, true, true>()),
             ilog_max(tile_lds_doubles<GroupedCfg1, false, true>(), tile_lds_doubles<GroupedCfg1, true, false>())));

template <class C>
__device__ __forceinline__ void grouped_tile(const GroupedDesc& d, int tm, int tn, double* smem) {
  if (d.ta) {
    if (d.tb) gemm_tile<C, true, true>(d.g, tm, tn, smem, false);
    else      gemm_tile<C, true, false>(d.g, tm, tn, smem, false);
  } else {
    if (d.tb) gemm_tile<C, false, true>(d.g, tm, tn, smem, false);
    else      gemm_tile<C, false, false>(d.g, tm, tn, smem, false);
  }
}

// The waves of workgroup b (on XCD b % 8) walk that XCD's sublist; the host makes the grid a
// multiple of 8, so each XCD has gridDim.x / 8 workgroups.
__device__ __forceinline__ void grouped_wave_tiles(const int8_t* plan, const GroupedDesc* descs,
                                                   const int4* tiles) {
  const int64_t* xoff = reinterpret_cast<const int64_t*>(plan + sizeof(PlanHeader));
  const int xcd = blockIdx.x % kXcds;
  const int per_xcd = gridDim.x / kXcds;
  const int local = blockIdx.x / kXcds;
  if (local >= per_xcd) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  constexpr int kWaves = kGroupedThreads / 64;
  const int64_t stride = (int64_t)per_xcd * kWaves;
  const int64_t end = xoff[xcd + 1];
  for (int64_t t = xoff[xcd] + (int64_t)local * kWaves + wave; t < end; t += stride) {
    const int4 e = tiles[t];
    const GroupedDesc& d = descs[e.x];
    const int64_t i0 = (int64_t)e.y * kWT, j0 = (int64_t)e.z * kWT;
    if (d.ta) {
      if (d.tb) wave_tile<true, true>(d.g, i0, j0, lane);
      else      wave_tile<true, false>(d.g, i0, j0, lane);
    } else {
      if (d.tb) wave_tile<false, true>(d.g, i0, j0, lane);
      else      wave_tile<false, false>(d.g, i0, j0, lane);
    }
  }
}

__global__ void __launch_bounds__(kGroupedThreads) __attribute__((amdgpu_waves_per_eu(4)))
grouped_kernel(const int8_t* plan) {
  __shared__ double smem[kGroupedLds];
  const PlanHeader* h = reinterpret_cast<const PlanHeader*>(plan);
  const GroupedDesc* descs = reinterpret_cast<const GroupedDesc*>(plan + h->desc_offset);
  const int4* tiles = reinterpret_cast<const int4*>(plan + h->tile_offset);
  if (h->kind == 1) {
    grouped_wave_tiles(plan, descs, tiles);
    return;
  }
  const int64_t n = h->num_tiles;
  for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
    const int4 e = tiles[t];
    const GroupedDesc& d = descs[e.x];
    if (d.tile_class == 0) grouped_tile<GroupedCfg0>(d, e.y, e.z, smem);
    else                   grouped_tile<GroupedCfg1>(d, e.y, e.z, smem);
  }
}

struct GroupedTileRef {
  double cost;
  int32_t gemm, tm, tn;
};

int grouped_tile_dims(int cls, int* mt, int* nt) {
  if (cls == 0) { *mt = GroupedCfg0::MT; *nt = GroupedCfg0::NT; return 0; }
  if (cls == 1) { *mt = GroupedCfg1::MT; *nt = GroupedCfg1::NT; return 0; }
  if (cls == kWaveClass) { *mt = kWT; *nt = kWT; return 0; }
  return -1;
}

bool is_notrans(char t) { return t == 'N' || t == 'n'; }
bool is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
int64_t max1(int64_t x) { return x > 1 ? x : 1; }

// Argument checks in dgemm argument order; 0 or the 1-based position of the first bad argument.
// Every kernel addresses the elements of one k-panel by 32-bit byte offsets from the panel origin
// (loads of up to 16 bytes). For the rows and k-indices inside the matrix those offsets must not
// wrap: at most (min(kt, k) - 1) * ld + tile_rows elements for an operand contiguous along its
// tile rows, (min(tile_rows, rows) - 1) * ld + kt for one contiguous along k. (Tile rows beyond
// the matrix may wrap: they read other data of the same storage and feed only outputs that are
// never stored.)
bool operand_offsets_fit(bool contig_k, int64_t tile_rows, int64_t rows, int64_t kt, int64_t k,
                         int64_t ld) {
  const int64_t span = contig_k ? ((tile_rows < rows ? tile_rows : rows) - 1) * ld + kt
                                : ((kt < k ? kt : k) - 1) * ld + tile_rows;
  return span * 8 + 16 <= ((int64_t)1 << 32);
}

bool panel_offsets_fit(bool ta, bool tb, int64_t mt, int64_t nt, int64_t kt, int64_t m, int64_t n,
                       int64_t k, int64_t lda, int64_t ldb) {
  return operand_offsets_fit(ta, mt, m, kt, k, lda) && operand_offsets_fit(!tb, nt, n, kt, k, ldb);
}

int check_args(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
               const double* C, int64_t ldc) {
  if (!is_notrans(transa) && !is_trans(transa)) return 1;
  if (!is_notrans(transb) && !is_trans(transb)) return 2;
  if (m < 0) return 3;
  if (n < 0) return 4;
  if (k < 0) return 5;
  const bool empty = (m == 0 || n == 0);
  const bool reads_ab = !empty && alpha != 0.0 && k != 0;
  const bool touches_c = !empty && !((alpha == 0.0 || k == 0) && beta == 1.0);
  const int64_t rows_a = is_notrans(transa) ? m : k;
  const int64_t rows_b = is_notrans(transb) ? k : n;
  if (reads_ab && A == nullptr) return 7;
  if (lda < max1(rows_a)) return 8;
  if (reads_ab && B == nullptr) return 9;
  if (ldb < max1(rows_b)) return 10;
  if (touches_c && C == nullptr) return 12;
  if (ldc < max1(m)) return 13;
  return 0;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Shape-driven choice. Tiles are dealt over the kCUs CUs, so a CU processes about
// ceil(tiles / kCUs) tiles, up to wgs_per_cu of them at a time. Its time is estimated as
//   tiles per CU * mt * nt * (k + overhead) / (efficiency * occupancy),
// where efficiency is the measured one for the transpose case, occupancy = (resident / wgs_per_cu)^(1/3)
// discounts a CU holding fewer workgroups than it could (less latency hiding), and the overhead of
// kTileOverheadK / resident k-steps stands for a tile's prologue and epilogue (old C read, C
// written), which co-resident workgroups partly overlap. The smallest estimate wins; ties go to
// the earlier entry.
// For k <= kShortK the GEMM is bound by the old C streaming through HBM rather than by the
// MFMAs, and the variants are ranked by their efficiency measured on such a shape (which already
// includes the epilogue). Variants with two k-groups are priced only on grids of at most one tile
// per CU, with an efficiency measured there (or none: then one replaces the chosen one-group
// variant of the same tile when the grid is a single round, below).
constexpr double kTileOverheadK = 128.0;
constexpr int64_t kShortK = 256;

// The model's estimate for one variant (in multiply-adds per CU at the variant's efficiency), or
// a negative value when the variant has no efficiency for this regime.
double tile_cost(const Variant& var, bool ta, bool tb, int64_t m, int64_t n, int64_t k) {
  const bool short_k = k <= kShortK;
  const int eff = short_k ? var.short_k_permil : var.eff_permil[ta][tb];
  if (eff <= 0) return -1.0;
  const int64_t tiles = ceil_div(m, var.mt) * ceil_div(n, var.nt);
  if (var.ks != 1 && tiles > kCUs) return -1.0;  // k-split tiles pay off on one round only
  const int64_t per_cu = ceil_div(tiles, kCUs);
  const int64_t resident = per_cu < var.wgs_per_cu ? per_cu : var.wgs_per_cu;
  const double occupancy = std::cbrt((double)resident / var.wgs_per_cu);
  const double overhead = short_k ? 0.0 : kTileOverheadK / resident;
  return (double)per_cu * var.mt * var.nt * ((double)k + overhead) / (eff * 1e-3 * occupancy);
}

// The variant of least estimate, and that estimate.
int pick_by_cost(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double* cost) {
  int best = 0;
  double best_cost = 0.0;
  for (int v = 0; v < kNumVariants; ++v) {
    const double c = tile_cost(kVariants[v], ta, tb, m, n, k);
    if (c < 0.0) continue;
    if (best_cost == 0.0 || c < best_cost) {
      best = v;
      best_cost = c;
    }
  }
  *cost = best_cost;
  return best;
}

// A grid of at most one workgroup per CU leaves each SIMD one wave of a one-group tile; the
// k-split configuration of the same tile runs two per SIMD there (measured at 1024^3: 8% faster;
// with two or more tiles per CU the one-group form is as fast or faster). Four groups (four waves
// per SIMD, two ring slots) pay off only on long k: on 64x64 tiles 2-5% faster than two groups at
// k = 4096 and 8192, the same at 2048, 1-5% slower at k = 300 to 1024.
constexpr int64_t kFourGroupsK = 2048;

int with_k_split(int v, int64_t m, int64_t n, int64_t k) {
  const Variant& b = kVariants[v];
  if (k > kShortK && b.ks == 1 && ceil_div(m, b.mt) * ceil_div(n, b.nt) <= kCUs) {
    int two = -1, four = -1;
    for (int w = 0; w < kNumVariants; ++w) {
      if (kVariants[w].mt != b.mt || kVariants[w].nt != b.nt) continue;
      if (kVariants[w].ks == 2) two = w;
      if (kVariants[w].ks == 4) four = w;
    }
    if (four >= 0 && k > kFourGroupsK) return four;
    if (two >= 0) return two;
  }
  return v;
}

int pick_variant(bool ta, bool tb, int64_t m, int64_t n, int64_t k) {
  double cost;
  return with_k_split(pick_by_cost(ta, tb, m, n, k, &cost), m, n, k);
}

// Plan of an automatic dgemm: the variant `vid` computes the block of rows [0, m0) and columns
// [0, n0) of C (vid = -1: no tiled block); the thin kernel computes rows [m0, m) over all
// columns and columns [n0, n) over rows [0, m0). Each thin side is at most kThinMax wide.
struct DgemmPlan {
  int vid;
  int64_t m0, n0;
};

// Estimates of the thin kernel in the model's units: its HBM bytes (the long operand once, C read
// and written) at kThinBytesPerSec plus one launch, converted at the CUs' multiply-add rate.
constexpr double kThinBytesPerSec = 4.0e12;
constexpr double kLaunchSec = 5e-6;
constexpr double kCuMacPerSec = 64.0 * 2.4e9;  // FP64 multiply-adds per second of one CU
// A fringe is split off only when the estimate drops by this factor (the model is coarse).
constexpr double kSplitGain = 0.95;

double thin_bytes(int64_t L, int64_t s, int64_t k) { return 8.0 * ((double)k * L + 2.0 * s * L); }

double thin_cost(double bytes) { return (bytes / kThinBytesPerSec + kLaunchSec) * kCuMacPerSec; }

DgemmPlan plan_dgemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k) {
  double best_cost;
  DgemmPlan best{pick_by_cost(ta, tb, m, n, k, &best_cost), m, n};
  if (m <= kThinMax || n <= kThinMax) {
    const bool rows = m <= n;  // the thinner side
    const double c = thin_cost(rows ? thin_bytes(n, m, k) : thin_bytes(m, n, k));
    if (c < best_cost) {
      best = rows ? DgemmPlan{-1, 0, n} : DgemmPlan{-1, m, 0};
      best_cost = c;
    }
  }
  // Big tiles over the largest block they divide, when what is left over is thin.
  DgemmPlan split{-1, m, n};
  double split_cost = 0.0;
  for (int v = 0; v < kNumVariants; ++v) {
    const Variant& var = kVariants[v];
    const int64_t rm = m % var.mt, rn = n % var.nt;
    const int64_t m0 = (rm != 0 && rm <= kThinMax && m > var.mt) ? m - rm : m;
    const int64_t n0 = (rn != 0 && rn <= kThinMax && n > var.nt) ? n - rn : n;
    if (m0 == m && n0 == n) continue;
    const double c0 = tile_cost(var, ta, tb, m0, n0, k);
    if (c0 < 0.0) continue;
    const double c = c0 + thin_cost((m0 < m ? thin_bytes(n, m - m0, k) : 0.0) +
                                    (n0 < n ? thin_bytes(m0, n - n0, k) : 0.0));
    if (split_cost == 0.0 || c < split_cost) {
      split = DgemmPlan{v, m0, n0};
      split_cost = c;
    }
  }
  if (split.vid >= 0 && split_cost < best_cost * kSplitGain) best = split;
  if (best.vid >= 0) best.vid = with_k_split(best.vid, best.m0, best.n0, k);
  return best;
}

thread_local int t_last_hip_error = 0;  // raw hipError_t of the last failed HIP call, per thread

int hip_fail(hipError_t e) {
  t_last_hip_error = (int)e;
  return MDG_ERR_HIP;
}

}  // namespace mdg_impl

void mdg_record_hip_error(int err) { mdg_impl::t_last_hip_error = err; }

namespace mdg_impl {

// Per-device memo of the architecture check (0 unknown, 1 gfx950, 2 other). Concurrent first
// calls may both query; they store the same value.
constexpr int kMaxDevices = 64;
std::atomic<int> g_arch_ok[kMaxDevices];

int device_check() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  int known = (dev >= 0 && dev < kMaxDevices) ? g_arch_ok[dev].load(std::memory_order_relaxed) : 0;
  if (known == 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e);
    known = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    if (dev >= 0 && dev < kMaxDevices) g_arch_ok[dev].store(known, std::memory_order_relaxed);
  }
  return known == 1 ? 0 : MDG_ERR_DEVICE;
}

// Launch and report this launch's own status (hipLaunchKernel's return value, not the
// thread's sticky last-error, which may hold an unrelated earlier failure).
template <typename... Args>
int launch(const void* fn, dim3 grid, dim3 block, hipStream_t s, Args... args) {
  void* argv[] = {static_cast<void*>(&args)...};
  hipError_t e = hipLaunchKernel(fn, grid, block, argv, 0, s);
  return e == hipSuccess ? MDG_SUCCESS : hip_fail(e);
}

// ---- symmetric rank-k update: host side ----------------------------------------------------------

bool is_lower(char u) { return u == 'L' || u == 'l'; }
bool is_upper(char u) { return u == 'U' || u == 'u'; }

int variant_by_name(const char* name) {
  for (int v = 0; v < kNumVariants; ++v)
    if (std::strcmp(kVariants[v].name, name) == 0) return v;
  return -1;
}

// Tiles of an n x n C with mt x nt tiles that meet one triangle (1 lower, 2 upper): tile row a
// of the lower triangle reaches tile column floor(((a+1) mt - 1) / nt), tile column b of the
// upper one tile row floor(((b+1) nt - 1) / mt), each cut at the edge.
int64_t syrk_tiles(int tri, int64_t n, int mt, int nt) {
  const int64_t along = tri == 1 ? mt : nt, across = tri == 1 ? nt : mt;
  const int64_t lines = ceil_div(n, along), width = ceil_div(n, across);
  int64_t total = 0;
  for (int64_t a = 0; a < lines; ++a) {
    const int64_t last = ((a + 1) * along - 1) / across;
    total += (last + 1 < width ? last + 1 : width);
  }
  return total;
}

// Workgroups of the launch: every tile of the super-tiles on one side of the diagonal.
int64_t syrk_workgroups(int64_t n, int mt, int nt, int side) {
  const int64_t lines = ceil_div(n, side);
  return lines * (lines + 1) / 2 * (side / mt) * (side / nt);
}

// The entry of kSyrkVariants with the smallest estimated time under the GEMM cost model
// (pick_variant) over the tiles that meet triangle `tri` in `batch` diagonal blocks of order n;
// `only` >= 0 restricts the choice to the entry named like kVariants[only]. Returns -1 if none
// qualifies.
int pick_syrk(int tri, bool ta, int64_t n, int64_t k, int only, int64_t batch = 1) {
  int best = -1;
  double best_cost = 0.0;
  const bool short_k = k <= kShortK;
  for (int s = 0; s < kNumSyrkVariants; ++s) {
    const SyrkVariant& sv = kSyrkVariants[s];
    const int vid = variant_by_name(sv.name);
    if (vid < 0 || (only >= 0 && vid != only)) continue;
    const Variant& var = kVariants[vid];
    int eff = short_k ? var.short_k_permil : var.eff_permil[ta][!ta];
    if (eff <= 0 && only >= 0) eff = 1;  // an explicit choice runs even if never automatic
    if (eff <= 0) continue;
    const int64_t tiles = batch * syrk_tiles(tri, n, var.mt, var.nt);
    const int64_t per_cu = ceil_div(tiles, kCUs);
    const int64_t resident = per_cu < var.wgs_per_cu ? per_cu : var.wgs_per_cu;
    const double occupancy = std::cbrt((double)resident / var.wgs_per_cu);
    const double overhead = short_k ? 0.0 : kTileOverheadK / resident;
    const double cost = (double)per_cu * var.mt * var.nt * ((double)k + overhead) /
                        (eff * 1e-3 * occupancy);
    if (best < 0 || cost < best_cost) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}

// dsyrk with n = kSyrkLeaf * 2^j >= kSyrkSplitN (automatic variant) is computed as diagonal
// blocks of order kSyrkLeaf plus the rectangles between them. Halving the range of blocks
// recursively, the lower (upper) rectangle of each halving is one GEMM, so most of the work runs
// as a few large square GEMMs at the GEMM's efficiency (at n = 8192: one 4096^2, two 2048^2 and
// four 1024^2 products with k = 8192 take 6.6 ms, 73 TFLOP/s); the diagonal blocks then run as one
// launch of the triangle kernel over all of them (blockIdx.y selects the block). Measured against
// the single triangle launch, k = n: n = 8192 7.9 against 8.6 ms, n = 4096 1.11 against 1.13 ms;
// at n = 6144 (six blocks, so rectangles of 2048 x 1024 and 3072 x 3072 that tile badly) 3.9
// against 3.6 ms, hence the restriction to powers of two. With k < 2048 the GEMMs are short and
// the extra launches cost more than they save (n = 8192: 3-18% slower at k = 40 to 1024, 1%
// faster at 2048; n = 4096: the same at 2048).
constexpr int64_t kSyrkSplitN = 4096;
constexpr int64_t kSyrkSplitK = 2048;
constexpr int64_t kSyrkLeaf = 1024;

bool syrk_splits(int64_t n, int64_t k) {
  if (n < kSyrkSplitN || k < kSyrkSplitK || n % kSyrkLeaf != 0) return false;
  const int64_t p = n / kSyrkLeaf;
  return (p & (p - 1)) == 0;
}

struct SyrkRect {
  int64_t r0, rows, c0, cols;
};

// The rectangles between diagonal blocks [l0, l1) of order nb of an n x n C, for triangle tri.
void syrk_rects(int tri, int64_t n, int64_t nb, int64_t l0, int64_t l1, std::vector<SyrkRect>& out) {
  if (l1 - l0 < 2) return;
  const int64_t mid = (l0 + l1) / 2;
  const int64_t lo = l0 * nb, mi = mid * nb, hi = std::min(l1 * nb, n);
  if (tri == 1) out.push_back(SyrkRect{mi, hi - mi, lo, mi - lo});  // rows below, columns left
  else out.push_back(SyrkRect{lo, mi - lo, mi, hi - mi});           // rows above, columns right
  syrk_rects(tri, n, nb, l0, mid, out);
  syrk_rects(tri, n, nb, mid, l1, out);
}

}  // namespace mdg_impl

using namespace mdg_impl;

extern "C" {

int mdg_version(void) { return kVersion; }

int mdg_last_hip_error(void) { return t_last_hip_error; }

int mdg_num_variants(void) { return kNumVariants; }

const char* mdg_variant_name(int variant) {
  return (variant >= 0 && variant < kNumVariants) ? kVariants[variant].name : nullptr;
}

int mdg_variant_info(int variant, int* mt, int* nt, int* kt, int* threads) {
  if (variant < 0 || variant >= kNumVariants) return MDG_ERR_VARIANT;
  const Variant& v = kVariants[variant];
  if (mt) *mt = v.mt;
  if (nt) *nt = v.nt;
  if (kt) *kt = v.kt;
  if (threads) *threads = v.threads;
  return 0;
}

const char* mdg_status_string(int status) {
  switch (status) {
    case MDG_SUCCESS: return "success";
    case 1: return "invalid argument 1: transa is not one of N, n, T, t, C, c";
    case 2: return "invalid argument 2: transb is not one of N, n, T, t, C, c";
    case 3: return "invalid argument 3: m < 0";
    case 4: return "invalid argument 4: n < 0";
    case 5: return "invalid argument 5: k < 0";
    case 7: return "invalid argument 7: A is NULL but would be read";
    case 8: return "invalid argument 8: lda < max(1, rows of stored A)";
    case 9: return "invalid argument 9: B is NULL but would be read";
    case 10: return "invalid argument 10: ldb < max(1, rows of stored B)";
    case 12: return "invalid argument 12: C is NULL but would be accessed";
    case 13: return "invalid argument 13: ldc < max(1, m)";
    case MDG_ERR_HIP: return "HIP runtime error";
    case MDG_ERR_VARIANT: return "unknown kernel variant";
    case MDG_ERR_DEVICE: return "current device is not gfx950";
    case MDG_ERR_SIZE: return "problem too large for one launch (grid size or leading dimension)";
    case MDG_ERR_SCRATCH: return "problem needs more scratch than the no-allocation entry point holds";
    default: return "unknown status";
  }
}

int mdg_select_variant(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                       double beta) {
  (void)beta;
  if (!(is_notrans(transa) || is_trans(transa)) || !(is_notrans(transb) || is_trans(transb)))
    return -1;
  if (m <= 0 || n <= 0 || k <= 0 || alpha == 0.0) return -1;
  return plan_dgemm(is_trans(transa), is_trans(transb), m, n, k).vid;
}

int mdg_dgemm_plan(char transa, char transb, int64_t m, int64_t n, int64_t k, int* variant,
                   int64_t* m_main, int64_t* n_main) {
  if (!(is_notrans(transa) || is_trans(transa))) return 1;
  if (!(is_notrans(transb) || is_trans(transb))) return 2;
  if (m <= 0) return 3;
  if (n <= 0) return 4;
  if (k <= 0) return 5;
  if (!variant) return 6;
  if (!m_main) return 7;
  if (!n_main) return 8;
  const DgemmPlan pl = plan_dgemm(is_trans(transa), is_trans(transb), m, n, k);
  *variant = pl.vid;
  *m_main = pl.vid >= 0 ? pl.m0 : 0;
  *n_main = pl.vid >= 0 ? pl.n0 : 0;
  return MDG_SUCCESS;
}

}  // extern "C"

namespace mdg_impl {

// Every check mdg_dgemm_ex makes before its first HIP call. Returns the status it would return
// there (nonzero), or 0 with *plan what to launch: plan->vid = -2 nothing; when alpha == 0 or
// k == 0 (and beta != 1) the scaling of C; otherwise the plan (an explicit variant covers all
// of C).
int dgemm_prepare(int variant, char transa, char transb, int64_t m, int64_t n, int64_t k,
                  double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double beta, const double* C, int64_t ldc, DgemmPlan* plan) {
  *plan = DgemmPlan{-2, m, n};
  const int info = check_args(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  if (info) return info;
  if (variant != MDG_VARIANT_AUTO && (variant < 0 || variant >= kNumVariants))
    return MDG_ERR_VARIANT;
  if (m == 0 || n == 0) return MDG_SUCCESS;
  const bool no_product = (alpha == 0.0 || k == 0);
  if (no_product && beta == 1.0) return MDG_SUCCESS;
  if (no_product) {
    *plan = DgemmPlan{-1, m, n};
    return MDG_SUCCESS;
  }
  const bool ta = is_trans(transa), tb = is_trans(transb);
  DgemmPlan pl =
      (variant == MDG_VARIANT_AUTO) ? plan_dgemm(ta, tb, m, n, k) : DgemmPlan{variant, m, n};
  // The thin launch's workgroups: 16 outputs each along n (fringe rows) and along m0 (fringe
  // columns). Offsets or a grid beyond the thin kernel's keep the whole product on the tiles.
  const int64_t thin_blocks = (pl.m0 < m ? ceil_div(n, kThinL) : 0) +
                              (pl.n0 < n && pl.m0 > 0 ? ceil_div(pl.m0, kThinL) : 0);
  if (thin_blocks > 0 &&
      (std::max(lda, ldb) > kThinMaxLd || thin_blocks > (int64_t)INT32_MAX / 1024))
    pl = DgemmPlan{pick_variant(ta, tb, m, n, k), m, n};
  if (pl.vid >= 0) {
    const Variant& v = kVariants[pl.vid];
    if (ceil_div(pl.m0, v.mt) * ceil_div(pl.n0, v.nt) > (int64_t)INT32_MAX / 1024)
      return MDG_ERR_SIZE;  // beyond one launch's grid
    if (!panel_offsets_fit(ta, tb, v.mt, v.nt, v.kt, pl.m0, pl.n0, k, lda, ldb))
      return MDG_ERR_SIZE;
  }
  *plan = pl;
  return MDG_SUCCESS;
}

}  // namespace mdg_impl

int mdg_dgemm_precheck(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                       const double* C, int64_t ldc) {
  DgemmPlan plan;
  return dgemm_prepare(MDG_VARIANT_AUTO, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                       ldc, &plan);
}

int mdg_device_check(void) { return device_check(); }

extern "C" {

int mdg_dgemm_ex(int variant, char transa, char transb, int64_t m, int64_t n, int64_t k,
                 double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                 double beta, double* C, int64_t ldc, void* stream) {
  DgemmPlan plan;
  const int st = dgemm_prepare(variant, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                               ldc, &plan);
  if (st || plan.vid == -2) return st;
  const int dc = device_check();
  if (dc) return dc;
  hipStream_t s = static_cast<hipStream_t>(stream);

  if (alpha == 0.0 || k == 0) {
    const int64_t total = m * n;
    const int64_t blocks = ceil_div(total, 256) < 65536 ? ceil_div(total, 256) : 65536;
    return launch(reinterpret_cast<const void*>(&scale_c_kernel), dim3((unsigned)blocks), dim3(256),
                  s, m, n, beta, C, ldc);
  }

  const bool ta = is_trans(transa), tb = is_trans(transb);
  if (plan.vid >= 0) {
    const int64_t mm = plan.m0, nn = plan.n0;
    const Variant& v = kVariants[plan.vid];
    const int64_t tiles_m = ceil_div(mm, v.mt), tiles_n = ceil_div(nn, v.nt);
    const int64_t tiles = tiles_m * tiles_n;
    const int64_t rows_a = ta ? k : mm, cols_a = ta ? mm : k;
    const int64_t rows_b = tb ? nn : k, cols_b = tb ? k : nn;
    GemmArgs g{mm, nn, k, lda, ldb, ldc, alpha, beta, A, B, C,
               (cols_a - 1) * lda + rows_a, (cols_b - 1) * ldb + rows_b};
    KernelFn fn = v.fn[ta ? 1 : 0][tb ? 1 : 0];
    const int64_t grid = (tiles + kXcds - 1) / kXcds * kXcds;  // see tile_coords
    const int r = launch(reinterpret_cast<const void*>(fn), dim3((unsigned)grid), dim3(v.threads),
                         s, g, (int)tiles_m, (int)tiles_n);
    if (r) return r;
  }

  // The thin fringes: rows [m0, m) over all columns, columns [n0, n) over rows [0, m0).
  ThinPair tp{};
  int parts = 0, side = 0;
  int64_t blocks = 0;
  if (plan.m0 < m) {  // op(A) rows m0.. times op(B)
    const int64_t r0 = plan.m0;
    tp.p[parts] = ThinArgs{m - r0, n, k,
                           B, tb ? ldb : 1, tb ? 1 : ldb,
                           ta ? A + r0 * lda : A + r0, ta ? lda : 1, ta ? 1 : lda,
                           C + r0, 1, ldc,
                           alpha, beta, tb ? 0 : 1, ta ? 1 : 0};
    side = std::max<int>(side, (int)(m - r0));
    blocks += ceil_div(n, kThinL);
    if (parts == 0) tp.blocks0 = (int)blocks;
    ++parts;
  }
  if (plan.n0 < n && plan.m0 > 0) {  // op(A) rows 0..m0 times op(B) columns n0..
    const int64_t c0 = plan.n0;
    tp.p[parts] = ThinArgs{n - c0, plan.m0, k,
                           A, ta ? 1 : lda, ta ? lda : 1,
                           tb ? B + c0 : B + c0 * ldb, tb ? 1 : ldb, tb ? ldb : 1,
                           C + c0 * ldc, ldc, 1,
                           alpha, beta, ta ? 1 : 0, tb ? 0 : 1};
    side = std::max<int>(side, (int)(n - c0));
    blocks += ceil_div(plan.m0, kThinL);
    if (parts == 0) tp.blocks0 = (int)blocks;
    ++parts;
  }
  if (parts == 0) return MDG_SUCCESS;
  const void* fn = side <= 4   ? reinterpret_cast<const void*>(&thin_kernel<4>)
                   : side <= 8 ? reinterpret_cast<const void*>(&thin_kernel<8>)
                               : reinterpret_cast<const void*>(&thin_kernel<16>);
  return launch(fn, dim3((unsigned)blocks), dim3(256), s, tp);
}

int mdg_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, void* stream) {
  return mdg_dgemm_ex(MDG_VARIANT_AUTO, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                      ldc, stream);
}

int mdg_dsyrk_ex(int variant, char uplo, char trans, int64_t n, int64_t k, double alpha,
                 const double* A, int64_t lda, double beta, double* C, int64_t ldc,
                 void* stream) {
  if (!is_lower(uplo) && !is_upper(uplo)) return 1;
  if (!is_notrans(trans) && !is_trans(trans)) return 2;
  if (n < 0) return 3;
  if (k < 0) return 4;
  const bool ta = is_trans(trans);
  const bool no_product = (alpha == 0.0 || k == 0);
  if (n > 0 && !no_product && A == nullptr) return 6;
  if (lda < max1(ta ? k : n)) return 7;
  const bool touches_c = n > 0 && !(no_product && beta == 1.0);
  if (touches_c && C == nullptr) return 9;
  if (ldc < max1(n)) return 10;
  if (variant != MDG_VARIANT_AUTO && (variant < 0 || variant >= kNumVariants))
    return MDG_ERR_VARIANT;
  if (!touches_c) return MDG_SUCCESS;
  const int tri = is_lower(uplo) ? 1 : 2;

  // Automatic calls on n = 1024 * 2^j >= 4096 with k >= 2048: the rectangles between diagonal
  // blocks as GEMMs, then one launch over the diagonal blocks (syrk_splits); otherwise one launch
  // over the whole triangle.
  const bool split = !no_product && variant == MDG_VARIANT_AUTO && syrk_splits(n, k);
  const int64_t leaf = split ? kSyrkLeaf : n;
  const int64_t blocks = split ? ceil_div(n, kSyrkLeaf) : 1;
  std::vector<SyrkRect> rects;
  const char op_a = ta ? 'T' : 'N', op_b = ta ? 'N' : 'T';
  auto a_at = [&](int64_t row) { return ta ? A + row * lda : A + row; };  // row of op(A)
  if (split) {
    syrk_rects(tri, n, leaf, 0, blocks, rects);
    for (const SyrkRect& r : rects) {  // every GEMM checked before anything is enqueued
      const int c = mdg_dgemm_precheck(op_a, op_b, r.rows, r.cols, k, alpha, a_at(r.r0), lda,
                                       a_at(r.c0), lda, beta, C + r.c0 * ldc + r.r0, ldc);
      if (c) return c;
    }
  }
  int s_idx = -1;
  int64_t wgs = 0;
  if (!no_product) {
    s_idx = pick_syrk(tri, ta, leaf, k, variant, blocks);
    if (s_idx < 0) return MDG_ERR_VARIANT;
    const SyrkVariant& sv = kSyrkVariants[s_idx];
    const Variant& v = kVariants[variant_by_name(sv.name)];
    wgs = syrk_workgroups(leaf, v.mt, v.nt, sv.super_side);
    if (wgs > (int64_t)INT32_MAX / 1024 || blocks > 65535) return MDG_ERR_SIZE;
    if (!panel_offsets_fit(ta, !ta, v.mt, v.nt, v.kt, n, n, k, lda, lda)) return MDG_ERR_SIZE;
  } else if (variant != MDG_VARIANT_AUTO && pick_syrk(tri, ta, n, 1024, variant) < 0) {
    return MDG_ERR_VARIANT;
  }
  const int dc = device_check();
  if (dc) return dc;
  hipStream_t s = static_cast<hipStream_t>(stream);

  if (no_product) {
    const int64_t blocks = ceil_div(n * n, 256) < 65536 ? ceil_div(n * n, 256) : 65536;
    return launch(reinterpret_cast<const void*>(&scale_tri_kernel), dim3((unsigned)blocks),
                  dim3(256), s, n, tri == 1 ? 1 : 0, beta, C, ldc);
  }
  for (const SyrkRect& r : rects) {
    const int st = mdg_dgemm_ex(MDG_VARIANT_AUTO, op_a, op_b, r.rows, r.cols, k, alpha,
                                a_at(r.r0), lda, a_at(r.c0), lda, beta, C + r.c0 * ldc + r.r0, ldc,
                                stream);
    if (st) return st;
  }
  const SyrkVariant& sv = kSyrkVariants[s_idx];
  const Variant& v = kVariants[variant_by_name(sv.name)];
  const int64_t rows_a = ta ? k : n, cols_a = ta ? n : k;
  const int64_t ext = (cols_a - 1) * lda + rows_a;
  GemmArgs g{n, n, k, lda, lda, ldc, alpha, beta, A, A, C, ext, ext};
  const int64_t grid = (wgs + kXcds - 1) / kXcds * kXcds;
  return launch(reinterpret_cast<const void*>(sv.fn[ta ? 1 : 0][tri == 1 ? 0 : 1]),
                dim3((unsigned)grid, (unsigned)blocks), dim3(v.threads), s, g, (int)wgs, leaf);
}

int mdg_dsyrk(char uplo, char trans, int64_t n, int64_t k, double alpha, const double* A,
              int64_t lda, double beta, double* C, int64_t ldc, void* stream) {
  return mdg_dsyrk_ex(MDG_VARIANT_AUTO, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream);
}

int mdg_dsyrk_select_variant(char uplo, char trans, int64_t n, int64_t k) {
  if ((!is_lower(uplo) && !is_upper(uplo)) || (!is_notrans(trans) && !is_trans(trans)) ||
      n < 0 || k < 0)
    return MDG_ERR_VARIANT;
  const bool split = syrk_splits(n, k);
  const int s_idx = pick_syrk(is_lower(uplo) ? 1 : 2, is_trans(trans), split ? kSyrkLeaf : n, k, -1,
                              split ? ceil_div(n, kSyrkLeaf) : 1);
  return s_idx < 0 ? MDG_ERR_VARIANT : variant_by_name(kSyrkVariants[s_idx].name);
}


// ---- grouped launch -----------------------------------------------------------------------------

// Tiles a GEMM contributes: none when nothing is computed (empty, or quick return).
static int64_t grouped_tiles_of(const mdg_gemm_desc& d, int cls) {
  if (d.m <= 0 || d.n <= 0) return 0;
  if ((d.alpha == 0.0 || d.k == 0) && d.beta == 1.0) return 0;
  int mt, nt;
  if (grouped_tile_dims(cls, &mt, &nt)) return 0;
  return ceil_div(d.m, mt) * ceil_div(d.n, nt);
}

static int grouped_class_of(const mdg_gemm_desc& d, const int32_t* tile_class, int i) {
  if (tile_class) return tile_class[i];
  return (d.m < 48 || d.n < 48) ? 1 : 0;
}

int mdg_grouped_tile_classes(void) { return kGroupedClasses; }

// Plan kind for these classes: 0 (classes 0 and 1 only), 1 (class 2 only), -1 (bad or mixed).
static int grouped_plan_kind(int count, const mdg_gemm_desc* descs, const int32_t* tile_class) {
  int wave = 0, block = 0;
  for (int i = 0; i < count; ++i) {
    const int cls = grouped_class_of(descs[i], tile_class, i);
    if (cls < 0 || cls >= kGroupedClasses) return -1;
    (cls == kWaveClass ? wave : block) += 1;
  }
  if (wave && block) return -1;
  return wave ? 1 : 0;
}

int64_t mdg_grouped_plan_bytes(int count, const mdg_gemm_desc* descs, const int32_t* tile_class) {
  if (count < 0 || (count > 0 && descs == nullptr)) return -1;
  const int kind = grouped_plan_kind(count, descs, tile_class);
  if (kind < 0) return -1;
  int64_t tiles = 0;
  for (int i = 0; i < count; ++i) tiles += grouped_tiles_of(descs[i], grouped_class_of(descs[i], tile_class, i));
  return (int64_t)sizeof(PlanHeader) + (kind ? kXcdTableBytes : 0) +
         (int64_t)count * (int64_t)sizeof(GroupedDesc) + tiles * 16;
}

int mdg_grouped_plan(int count, const mdg_gemm_desc* descs, const int32_t* tile_class,
                     int schedule, void* plan, int64_t plan_bytes, int64_t* num_tiles,
                     int* bad_index) {
  if (bad_index) *bad_index = -1;
  if (count < 0 || (count > 0 && descs == nullptr)) return 1;
  if (schedule != MDG_SCHEDULE_NATURAL && schedule != MDG_SCHEDULE_LPT) return 4;
  const int64_t need = mdg_grouped_plan_bytes(count, descs, tile_class);
  if (need < 0) return 3;
  if (plan == nullptr || plan_bytes < need) return 5;
  const int kind = grouped_plan_kind(count, descs, tile_class);
  std::vector<GroupedTileRef> refs;
  int8_t* base = static_cast<int8_t*>(plan);
  PlanHeader* h = reinterpret_cast<PlanHeader*>(base);
  GroupedDesc* gd = reinterpret_cast<GroupedDesc*>(base + sizeof(PlanHeader) +
                                                   (kind ? kXcdTableBytes : 0));
  for (int i = 0; i < count; ++i) {
    const mdg_gemm_desc& d = descs[i];
    const int info = check_args(d.transa, d.transb, d.m, d.n, d.k, d.alpha, d.A, d.lda, d.B, d.ldb,
                                d.beta, d.C, d.ldc);
    if (info) {
      if (bad_index) *bad_index = i;
      return 100 + info;
    }
    const int cls = grouped_class_of(d, tile_class, i);
    int mt = 0, nt = 0;
    grouped_tile_dims(cls, &mt, &nt);
    const bool ta = is_trans(d.transa), tb = is_trans(d.transb);
    const int64_t rows_a = ta ? d.k : d.m, cols_a = ta ? d.m : d.k;
    const int64_t rows_b = tb ? d.n : d.k, cols_b = tb ? d.k : d.n;
    GroupedDesc& o = gd[i];
    std::memset(&o, 0, sizeof(o));
    o.g = GemmArgs{d.m, d.n, d.k, d.lda, d.ldb, d.ldc, d.alpha, d.beta, d.A, d.B, d.C,
                   cols_a > 0 ? (cols_a - 1) * d.lda + rows_a : 0,
                   cols_b > 0 ? (cols_b - 1) * d.ldb + rows_b : 0};
    o.ta = ta;
    o.tb = tb;
    o.tile_class = cls;
    const int64_t ntiles = grouped_tiles_of(d, cls);
    o.tiles_m = ntiles ? (int32_t)ceil_div(d.m, mt) : 0;
    o.tiles_n = ntiles ? (int32_t)ceil_div(d.n, nt) : 0;
    if (ntiles && (o.tiles_m > INT32_MAX / 2 || o.tiles_n > INT32_MAX / 2 ||
                   (d.alpha != 0.0 && d.k > 0 &&
                    !panel_offsets_fit(ta, tb, mt, nt, cls == kWaveClass ? kWK : 16, d.m, d.n,
                                       d.k, d.lda, d.ldb)))) {
      if (bad_index) *bad_index = i;
      return MDG_ERR_SIZE;
    }
    const double cost = (double)mt * nt * (double)(d.alpha == 0.0 ? 1 : (d.k > 0 ? d.k : 1));
    for (int32_t tn = 0; tn < o.tiles_n; ++tn)
      for (int32_t tm = 0; tm < o.tiles_m; ++tm) refs.push_back(GroupedTileRef{cost, i, tm, tn});
  }
  int64_t xoff[kXcds + 1] = {0};
  if (kind == 0) {
    if (schedule == MDG_SCHEDULE_LPT)
      std::stable_sort(refs.begin(), refs.end(), [](const GroupedTileRef& a, const GroupedTileRef& b) {
        return a.cost > b.cost;
      });
  } else {
    // Whole GEMMs to XCDs: LPT takes the GEMMs by decreasing total cost and gives each to the XCD
    // with the least work so far; NATURAL deals them round-robin in order. Each XCD's sublist then
    // holds its GEMMs in that order, each GEMM's tiles column by column.
    std::vector<double> gcost(count, 0.0);
    std::vector<int64_t> gfirst(count, -1), gcount(count, 0);
    for (size_t t = 0; t < refs.size(); ++t) {
      const int gi = refs[t].gemm;
      if (gfirst[gi] < 0) gfirst[gi] = (int64_t)t;
      gcount[gi] += 1;
      gcost[gi] += refs[t].cost;
    }
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    if (schedule == MDG_SCHEDULE_LPT)
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int b) { return gcost[a] > gcost[b]; });
    std::vector<int> owner(count, 0);
    double load[kXcds] = {0.0};
    int next = 0;
    for (int gi : order) {
      if (gcount[gi] == 0) continue;
      int x = 0;
      if (schedule == MDG_SCHEDULE_LPT) {
        for (int y = 1; y < kXcds; ++y)
          if (load[y] < load[x]) x = y;
      } else {
        x = next;
        next = (next + 1) % kXcds;
      }
      owner[gi] = x;
      load[x] += gcost[gi];
    }
    std::vector<GroupedTileRef> sorted;
    sorted.reserve(refs.size());
    for (int x = 0; x < kXcds; ++x) {
      xoff[x] = (int64_t)sorted.size();
      for (int gi : order)
        if (gcount[gi] > 0 && owner[gi] == x)
          for (int64_t t = 0; t < gcount[gi]; ++t) sorted.push_back(refs[gfirst[gi] + t]);
    }
    xoff[kXcds] = (int64_t)sorted.size();
    refs.swap(sorted);
  }
  h->magic = kPlanMagic;
  h->version = 2;
  h->count = count;
  h->kind = kind;
  h->num_tiles = (int64_t)refs.size();
  h->desc_offset = (int64_t)sizeof(PlanHeader) + (kind ? kXcdTableBytes : 0);
  h->tile_offset = h->desc_offset + (int64_t)count * (int64_t)sizeof(GroupedDesc);
  h->pad2[0] = h->pad2[1] = h->pad2[2] = 0;
  if (kind) {
    int64_t* xt = reinterpret_cast<int64_t*>(base + sizeof(PlanHeader));
    std::memset(xt, 0, kXcdTableBytes);
    for (int x = 0; x <= kXcds; ++x) xt[x] = xoff[x];
  }
  int32_t* tl = reinterpret_cast<int32_t*>(base + h->tile_offset);
  for (size_t t = 0; t < refs.size(); ++t) {
    tl[4 * t + 0] = refs[t].gemm;
    tl[4 * t + 1] = refs[t].tm;
    tl[4 * t + 2] = refs[t].tn;
    tl[4 * t + 3] = 0;
  }
  if (num_tiles) *num_tiles = (int64_t)refs.size();
  return MDG_SUCCESS;
}

int mdg_dgemm_grouped(const void* device_plan, int64_t num_tiles, int grid, void* stream) {
  if (device_plan == nullptr) return 1;
  if (num_tiles < 0) return 2;
  if (grid < 0) return 3;
  if ((reinterpret_cast<uintptr_t>(device_plan) & 15) != 0) return 1;
  if (num_tiles == 0) return MDG_SUCCESS;
  const int dc = device_check();
  if (dc) return dc;
  int64_t g = grid > 0 ? grid : (int64_t)kCUs * 4;
  if (g > num_tiles) g = num_tiles;
  g = (g + kXcds - 1) / kXcds * kXcds;  // wave-tile plans deal whole workgroups per XCD
  const int8_t* p = static_cast<const int8_t*>(device_plan);
  return launch(reinterpret_cast<const void*>(&grouped_kernel), dim3((unsigned)g),
                dim3(kGroupedThreads), static_cast<hipStream_t>(stream), p);
}

}  // extern "C"
