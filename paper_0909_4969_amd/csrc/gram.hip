// Gram matrices of matricizations, on the smaller side (the leading left
// singular vectors of a matrix M are the top eigenvectors of M M^T; when M
// has fewer columns than rows, they are M v / sigma for the top
// eigenvectors v of M^T M).
//
// A matricization M (rows i < I, columns j < J) of a C-order array with
// "inner size" Q (the product of the dimensions after the row mode) puts
// element (i, j) at  off(j) + i * Q,  off(j) = (j / Q) * I * Q + j mod Q.
// This covers both the HOOI intermediates Y_k (view O x I_k x Q) and the
// sampled tensor's unfolding Xhat_(n) (Q = stride of mode n).
//   row side:    G[x, y] = sum_j M[x, j] M[y, j]   (I x I)
//   column side: G[x, y] = sum_i M[i, x] M[i, y]   (J x J)
// Products are float32, summed in float32 over 32 terms and then in
// float64; each workgroup owns a 64x64 tile and a slice of the summation
// range, and the slices are added in a fixed order.
#include <algorithm>

#include "solver.h"

namespace mach {
namespace {

struct GramArgs {
  uint32_t I, Q, J;       // matricization shape and inner size
  FastDiv fQ;
  int kside;              // 1: column side (J x J), 0: row side (I x I)
  uint32_t X, Z;          // Gram side and summation length
  uint32_t zchunk;        // summation slice per workgroup
  double* part;           // [X][X][chunk] (chunk-minor)
  uint32_t nz;            // number of slices (chunks)
  const int32_t* st_solver;
  const SampleHdr* hdr;
};

struct DenseLoad {
  const float* base;
  __device__ __forceinline__ float operator()(uint32_t l) const { return base[l]; }
};

// Xhat (unscaled) at linear index l: bitmap test, rank, kept value.
struct MaskedLoad {
  const uint64_t* bitmap;
  const uint32_t* wrank;
  const Entry* coo;
  __device__ __forceinline__ float operator()(uint32_t l) const {
    uint64_t word = bitmap[l >> 6];
    uint32_t b = l & 63;
    if (!((word >> b) & 1ull)) return 0.f;
    uint64_t below = b ? (word & ((~0ull) >> (64 - b))) : 0ull;
    return coo[wrank[l >> 6] + (uint32_t)__popcll(below)].v;
  }
};

__device__ __forceinline__ uint32_t col_off(const GramArgs& a, uint32_t j) {
  uint32_t q = a.fQ.div(j);
  return q * a.I * a.Q + (j - q * a.Q);
}

template <typename Load>
__global__ __launch_bounds__(256) void k_gram(GramArgs a, Load ld) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  __shared__ float Mx[32][65];
  __shared__ float My[32][65];
  const uint32_t x0 = blockIdx.x * 64, y0 = blockIdx.y * 64;
  const uint32_t zb = blockIdx.z;
  const uint32_t zc0 = zb * a.zchunk;
  const uint32_t zc1 = min(a.Z, zc0 + a.zchunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // diagonal tiles (x0 == y0) stage one matrix; the next 32 summation
  // indices are loaded into registers while the current ones are used
  const bool same = x0 == y0;
  auto fetch = [&](uint32_t zs, float* px, float* py) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + 256 * u, zz = e >> 6, xx = e & 63;
      const uint32_t z = zs + zz;
      float vx = 0.f, vy = 0.f;
      if (z < zc1) {
        const uint32_t x = x0 + xx, y = y0 + xx;
        if (a.kside) {
          const uint32_t zo = z * a.Q;
          if (x < a.X) vx = ld(zo + col_off(a, x));
          if (!same && y < a.X) vy = ld(zo + col_off(a, y));
        } else {
          const uint32_t zo = col_off(a, z);
          if (x < a.X) vx = ld(zo + x * a.Q);
          if (!same && y < a.X) vy = ld(zo + y * a.Q);
        }
      }
      px[u] = vx;
      py[u] = vy;
    }
  };
  float px[8], py[8];
  fetch(zc0, px, py);
  for (uint32_t zs = zc0; zs < zc1; zs += 32) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + 256 * u;
      Mx[e >> 6][e & 63] = px[u];
      if (!same) My[e >> 6][e & 63] = py[u];
    }
    __syncthreads();
    if (zs + 32 < zc1) fetch(zs + 32, px, py);
    float (*Ny)[65] = same ? Mx : My;
    float c[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) c[i][j] = 0.f;
#pragma unroll 8
    for (int zz = 0; zz < 32; ++zz) {
      float u[4], w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        u[i] = Mx[zz][tx * 4 + i];
        w[i] = Ny[zz][ty * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c[i][j] = fmaf(u[i], w[j], c[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += (double)c[i][j];
    __syncthreads();
  }
  double* out = a.part;   // chunk-minor: entry (x, y) of slice zb
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t x = x0 + tx * 4 + i, y = y0 + ty * 4 + j;
      if (x < a.X && y < a.X) out[((size_t)x * a.X + y) * a.nz + zb] = acc[i][j];
    }
}

// G = sum over chunks of part (chunk-minor, fixed order).
__global__ void k_gram_reduce(const double* __restrict__ part, uint32_t nchunk, uint32_t n2,
                              double* __restrict__ G, const SampleHdr* hdr, const int32_t* st_solver) {
  if (hdr->status != 0 || *st_solver != 0) return;
  uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n2) return;
  const double* p = part + (size_t)e * nchunk;
  double s = 0.0;
#pragma unroll 8
  for (uint32_t c = 0; c < nchunk; ++c) s += p[c];
  G[e] = s;
}

template <typename Load>
hipError_t gram_run(GramArgs a, Load ld, double* G, size_t part_elems, hipStream_t st) {
  uint32_t tiles = (a.X + 63) / 64;
  uint64_t n2 = (uint64_t)a.X * a.X;
  // Slices of at least 256 summation indices; enough workgroups to fill
  // the chip; the partials must fit their buffer.
  uint32_t nchunk = 1;
  while (nchunk < 1024 && (uint64_t)tiles * tiles * nchunk < 512 &&
         a.Z / (2 * nchunk) >= 256 && n2 * (2 * nchunk) <= part_elems)
    nchunk *= 2;
  a.zchunk = (a.Z + nchunk - 1) / nchunk;
  a.zchunk = (a.zchunk + 31) / 32 * 32;
  nchunk = (a.Z + a.zchunk - 1) / a.zchunk;
  if (nchunk < 1) nchunk = 1;
  if (nchunk == 1) a.part = G;
  a.nz = nchunk;
  hipLaunchKernelGGL((k_gram<Load>), dim3(tiles, tiles, nchunk), dim3(256), 0, st, a, ld);
  if (nchunk > 1)
    hipLaunchKernelGGL(k_gram_reduce, dim3((uint32_t)((n2 + 255) / 256)), dim3(256), 0, st, a.part,
                       nchunk, (uint32_t)n2, G, a.hdr, a.st_solver);
  return hipGetLastError();
}

// Column-side Gram of the sampled unfolding when the mode is the single
// tail mode: G[r][r'] = sum_c Xhat[r, c] Xhat[r', c] over the CSR rows r
// (head rows) and tail columns c.  The CSC columns list their entries in
// the head order of the CSC layout (position headpos[r]); the entry (r, c)
// itself sits at the CSC position the layout build recorded (cscpos).  Each
// pair of entries of a column is taken once, by one of its two rows: in an
// even column by the row that comes first in head order (the entries from
// (r, c) to the column's end), in an odd column by the row that comes last
// (the entries from the column's start to (r, c)).  Every row then does
// about the same work, half a column per entry, wherever it sits in head
// order.  One wave per row r walks the row's entries (c, v) in order; for
// each, its lanes take the entries (r', v') of its part of column c and add
// v v' to a float64 accumulator of row r in LDS.  The entries of one column
// have distinct r', so lanes never collide, and every accumulator is summed
// in column order.  Row r writes its whole accumulator row: G[r][r'] then
// holds the even columns' sum when r comes first, the odd columns' sum when
// r comes last, and k_gram_mirror adds the two halves of every pair.
// Row r = v / 2 for even wave index v and MH - 1 - v / 2 for odd v.
//
// The walk is bound by its reads of the column lists, so the row's entries
// go in groups of kSgU and the first kSgC 64-entry chunks of every part in
// a group are loaded, unconditionally, before any is added (a part of a
// column of up to 256 entries needs no further load; longer ones finish in
// a loop).  The additions are plain LDS reads and writes, no atomics: the
// wave owns its accumulator row, the lanes of one part never share a row
// r', and LDS operations of one wave complete in the order they are issued,
// so every accumulator takes its terms in column order; each product v v'
// of two float32 values is exact in float64.  (With float64 LDS atomic
// adds in their place the kernel took 12 % longer.)
constexpr int kSgU = 4, kSgC = 4;

__global__ __launch_bounds__(256) void k_gram_rows_sparse(uint32_t MH, FastDiv fMT,
                                                          const uint32_t* __restrict__ headpos,
                                                          const Entry* __restrict__ coo_l,
                                                          const uint32_t* __restrict__ rowptr,
                                                          const Entry* __restrict__ coo_t,
                                                          const uint32_t* __restrict__ colptr,
                                                          const uint32_t* __restrict__ cscpos,
                                                          double* __restrict__ G, const SampleHdr* hdr,
                                                          const int32_t* st_solver) {
  if (hdr->status != 0 || *st_solver != 0) return;
  __shared__ double acc[4][kSparseGramMaxRows];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t v = blockIdx.x * 4 + w;
  const uint32_t r = (v & 1) ? MH - 1 - (v >> 1) : (v >> 1);
  double* row = acc[w];
  for (uint32_t j = lane; j < MH; j += 64) row[j] = 0.0;
  __builtin_amdgcn_wave_barrier();
  if (v < MH) {
    const uint32_t base = r * fMT.d;
    const uint32_t e1 = rowptr[r + 1];
    for (uint32_t e0 = rowptr[r]; e0 < e1; e0 += 64) {
      // lane i holds the descriptor of entry e0 + i: value, first and end
      // position of its part of the column
      const uint32_t e = e0 + lane;
      uint32_t lo = 0, hi = 0;
      float va = 0.0f;
      if (e < e1) {
        const Entry a = coo_l[e];
        const uint32_t c = a.l - base;
        va = a.v;
        lo = cscpos[e];
        if (c & 1u) {
          hi = lo + 1;
          lo = colptr[c];
        } else {
          hi = colptr[c + 1];
        }
      }
      const int cnt = (int)min(64u, e1 - e0);
      for (int k = 0; k < cnt; k += kSgU) {
        Entry b[kSgC][kSgU];
        uint32_t f[kSgU], h[kSgU];
        double vk[kSgU];
#pragma unroll
        for (int u = 0; u < kSgU; ++u) {
          const int ku = min(k + u, cnt - 1);
          f[u] = (uint32_t)__builtin_amdgcn_readlane((int)lo, ku) + lane;
          h[u] = k + u < cnt ? (uint32_t)__builtin_amdgcn_readlane((int)hi, ku) : 0u;
          vk[u] = (double)__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, va), ku));
          // Unconditional loads (a predicated load is compiled to a branch
          // that waits for it): lanes past the part read its last entry, or
          // entry 0 where the group has no entry u (the row's own entries
          // make the list non-empty); their terms are not added.
          const uint32_t last = h[u] > 0u ? h[u] - 1u : 0u;
#pragma unroll
          for (int j = 0; j < kSgC; ++j) b[j][u] = coo_t[min(f[u] + 64u * j, last)];
        }
#pragma unroll
        for (int u = 0; u < kSgU; ++u) {
          // The chunks of part u hold distinct rows r', so all their
          // accumulators are read first (every lane, at the row of its
          // entry, an index inside the row) and then written by the lanes
          // that hold an entry; the next part's reads come after these
          // writes in the wave's LDS order.
          uint32_t ix[kSgC];
          double cur[kSgC];
#pragma unroll
          for (int j = 0; j < kSgC; ++j) {
            ix[j] = fMT.div(b[j][u].l);
            cur[j] = row[ix[j]];
          }
#pragma unroll
          for (int j = 0; j < kSgC; ++j)
            if (f[u] + 64u * j < h[u]) row[ix[j]] = cur[j] + vk[u] * (double)b[j][u].v;
          for (uint32_t g = f[u] + 64u * kSgC; g < h[u]; g += 64) {
            const Entry e = coo_t[g];
            const uint32_t i = fMT.div(e.l);
            row[i] = row[i] + vk[u] * (double)e.v;
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t j = lane; j < MH; j += 64) G[(size_t)r * MH + j] = row[j];
  }
}

// Completes the Gram left by k_gram_rows_sparse: for x before y in head
// order G[x][y] holds the even columns' sum and G[y][x] the odd columns';
// both become their sum, added in that order (so the result is exactly
// symmetric).  The diagonal is already whole.  By pairs of 64 x 64 tiles
// (bi, bj) and (bj, bi), bi >= bj, through LDS.
__global__ __launch_bounds__(256) void k_gram_mirror(uint32_t MH, const uint32_t* __restrict__ headpos,
                                                     double* __restrict__ G, const SampleHdr* hdr,
                                                     const int32_t* st_solver) {
  if (hdr->status != 0 || *st_solver != 0) return;
  __shared__ double ta[64][65], tb[64][65];
  __shared__ uint32_t pi_[64], pj[64];
  const uint32_t bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  if (threadIdx.x < 64) {
    const uint32_t i = bi * 64 + threadIdx.x, j = bj * 64 + threadIdx.x;
    pi_[threadIdx.x] = i < MH ? headpos[i] : 0u;
    pj[threadIdx.x] = j < MH ? headpos[j] : 0u;
  }
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const uint32_t x = e >> 6, y = e & 63;
    const uint32_t ar = bi * 64 + x, ac = bj * 64 + y, br = bj * 64 + x, bc = bi * 64 + y;
    ta[x][y] = (ar < MH && ac < MH) ? G[(size_t)ar * MH + ac] : 0.0;
    tb[x][y] = (br < MH && bc < MH) ? G[(size_t)br * MH + bc] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const uint32_t x = e >> 6, y = e & 63;
    const uint32_t ar = bi * 64 + x, ac = bj * 64 + y;
    if (ar < MH && ac < MH && ar != ac) {
      const double own = ta[x][y], tr = tb[y][x];
      G[(size_t)ar * MH + ac] = pi_[x] < pj[y] ? own + tr : tr + own;
    }
    const uint32_t br = bj * 64 + x, bc = bi * 64 + y;
    if (bi != bj && br < MH && bc < MH) {
      const double own = tb[x][y], tr = ta[y][x];
      G[(size_t)br * MH + bc] = pj[x] < pi_[y] ? own + tr : tr + own;
    }
  }
}

// ---------------------------------------------------------------------------
// Row-side Gram of the sampled unfolding on MFMA (float32 products, float32
// accumulation over one chunk of columns, then float64).  Applies when the
// unfolding's rows are 64-aligned runs of the linear index (Q a multiple of
// 64), so that 64 columns of one row are one bitmap word and the kept
// values of that word are consecutive entries of the l-ordered list.
//
// The I x I Gram is cut into RB x RB blocks; workgroup (blk, slice) owns
// the upper-triangle block pair blk = (bx, by), bx <= by, and a slice of the
// columns.  Per chunk of CW = 4096 / RB columns it expands both row blocks
// of Xhat into LDS (dense float32, zeros where not kept), then its four
// waves take every fourth group of 4 columns and issue
// v_mfma_f32_16x16x4f32 on all (RB/16)^2 16x16 tiles.  The wave sums are
// added in a fixed order and the block partial is written to
// part[slice][blk]; a second kernel adds the slices in order and fills both
// triangles.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

struct MfmaGramArgs {
  const uint64_t* bitmap;
  const uint32_t* wrank;
  const Entry* coo;
  uint32_t I, Q, J;
  FastDiv fQ;
  uint32_t nb, nblk;       // row blocks, block pairs (nb (nb + 1) / 2)
  uint32_t cps;            // chunks per slice
  double* part;            // [slice][blk][RB][RB]
  const SampleHdr* hdr;
  const int32_t* st_solver;
};

// Staging of one chunk (RB rows x CW = 4096 / RB columns of Xhat_(n)).
// Each thread owns one bitmap word and 16 of its bits: the word's kept
// values are consecutive entries of the l-ordered list from the word's
// rank.  Two column layouts:
//  - Q1 = false (Q a multiple of 64): 64 consecutive columns of one row are
//    one word; thread (row r, word wd, quarter q).
//  - Q1 = true (the last mode, Q = 1, I a multiple of 64, RB = 64): the 64
//    rows of one column are one word; thread (column cc, quarter q).
template <int RB, bool Q1>
struct MfmaStage {
  static constexpr int CW = 4096 / RB;
  uint64_t word;
  uint32_t base;
  float v[16];

  __device__ __forceinline__ void load_word(const MfmaGramArgs& a, uint32_t row0, uint32_t jc) {
    const int t = threadIdx.x;
    word = 0;
    base = 0;
    if constexpr (Q1) {
      const uint32_t j = jc + (t >> 2);
      if (j < a.J && row0 < a.I) {
        const uint32_t l0 = j * a.I + row0;
        word = a.bitmap[l0 >> 6];
        base = a.wrank[l0 >> 6];
      }
    } else {
      constexpr int WPR = CW / 64;
      const int rw = t >> 2, r = rw / WPR, wd = rw % WPR;
      const uint32_t i = row0 + r, j = jc + wd * 64;
      if (i < a.I && j < a.J) {
        const uint32_t qq = a.fQ.div(j);
        const uint32_t l0 = qq * a.I * a.Q + (j - qq * a.Q) + i * a.Q;
        word = a.bitmap[l0 >> 6];
        base = a.wrank[l0 >> 6];
      }
    }
  }
  __device__ __forceinline__ void load_values(const MfmaGramArgs& a) {
    const int q = threadIdx.x & 3;
    const uint32_t below = (uint32_t)__popcll(q ? (word & ((~0ull) >> (64 - 16 * q))) : 0ull);
    const uint32_t bits = (uint32_t)(word >> (16 * q)) & 0xffffu;
    uint32_t r = base + below;
#pragma unroll
    for (int bb = 0; bb < 16; ++bb) {
      const bool kept = (bits >> bb) & 1u;
      v[bb] = kept ? a.coo[r].v : 0.f;
      r += kept ? 1u : 0u;
    }
  }
  __device__ __forceinline__ void store(float (*M)[CW + 4]) const {
    const int t = threadIdx.x, q = t & 3;
    if constexpr (Q1) {
      const int cc = t >> 2;
#pragma unroll
      for (int bb = 0; bb < 16; ++bb) M[q * 16 + bb][cc] = v[bb];
    } else {
      constexpr int WPR = CW / 64;
      const int rw = t >> 2, r = rw / WPR, wd = rw % WPR;
#pragma unroll
      for (int bb = 0; bb < 16; ++bb) M[r][wd * 64 + q * 16 + bb] = v[bb];
    }
  }
};

// Tiles of an RB x RB block: TB x TB 16 x 16 tiles.  With at least four
// tiles every wave owns a quarter of them over all columns; a single tile
// (RB = 16) is shared by the four waves, each taking every fourth group of
// 4 columns, and their sums are added in wave order.
template <int RB, bool Q1>
__global__ __launch_bounds__(256) void k_gram_mfma(MfmaGramArgs a) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  constexpr int CW = 4096 / RB, TB = RB / 16, KS = CW / 4;
  constexpr int NT = TB * TB, TPW = NT >= 4 ? NT / 4 : 1, KSPLIT = NT >= 4 ? 1 : 4;
  __shared__ float Ma[RB][CW + 4];
  __shared__ float Mb[RB][CW + 4];
  uint32_t by = 0;
  while ((by + 1) * (by + 2) / 2 <= blockIdx.x) ++by;
  const uint32_t bx = blockIdx.x - by * (by + 1) / 2;
  const bool diag = bx == by;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  v4f acc[TPW];
  double dacc[TPW][4];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) dacc[u][v] = 0.0;
  }
  const uint32_t c0 = blockIdx.y * a.cps;
  uint32_t c1 = c0 + a.cps;
  const uint32_t nchunk = (a.J + CW - 1) / CW;
  if (c1 > nchunk) c1 = nchunk;
  // Software pipeline: the values of chunk c + 1 and the words of chunk
  // c + 2 are requested while chunk c is multiplied.
  MfmaStage<RB, Q1> sa, sb;
  uint64_t wa2 = 0, wb2 = 0;
  uint32_t ba2 = 0, bb2 = 0;
  if (c0 < c1) {
    sa.load_word(a, bx * RB, c0 * CW);
    if (!diag) sb.load_word(a, by * RB, c0 * CW);
    sa.load_values(a);
    if (!diag) sb.load_values(a);
    if (c0 + 1 < c1) {
      MfmaStage<RB, Q1> t;
      t.load_word(a, bx * RB, (c0 + 1) * CW);
      wa2 = t.word;
      ba2 = t.base;
      if (!diag) {
        t.load_word(a, by * RB, (c0 + 1) * CW);
        wb2 = t.word;
        bb2 = t.base;
      }
    }
  }
  for (uint32_t c = c0; c < c1; ++c) {
    __syncthreads();
    sa.store(Ma);
    if (!diag) sb.store(Mb);
    __syncthreads();
    if (c + 1 < c1) {
      sa.word = wa2;
      sa.base = ba2;
      sa.load_values(a);
      if (!diag) {
        sb.word = wb2;
        sb.base = bb2;
        sb.load_values(a);
      }
      if (c + 2 < c1) {
        MfmaStage<RB, Q1> t;
        t.load_word(a, bx * RB, (c + 2) * CW);
        wa2 = t.word;
        ba2 = t.base;
        if (!diag) {
          t.load_word(a, by * RB, (c + 2) * CW);
          wb2 = t.word;
          bb2 = t.base;
        }
      }
    }
    float (*B)[CW + 4] = diag ? Ma : Mb;
    for (int ks = (KSPLIT > 1 ? w : 0); ks < KS; ks += KSPLIT) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int t = (NT >= 4 ? w * TPW : 0) + u, x = t / TB, y = t % TB;
        const float av = Ma[x * 16 + li][ks * 4 + lk];
        const float bv = B[y * 16 + li][ks * 4 + lk];
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[u], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[u][v] += (double)acc[u][v];
      acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  // Tiles to LDS (reusing the staging buffers): each wave writes its own
  // tiles; a shared tile is added up in wave order 0..3.
  __syncthreads();
  double* red = reinterpret_cast<double*>(&Ma[0][0]);
  static_assert(sizeof(Ma) + sizeof(Mb) >= RB * RB * sizeof(double), "reduction buffer");
  for (int ww = 0; ww < KSPLIT; ++ww) {
    if (KSPLIT == 1 || w == ww) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int t = (NT >= 4 ? w * TPW : 0) + u, x = t / TB, y = t % TB;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = x * 16 + lk * 4 + v, col = y * 16 + li;
          double* p = red + row * RB + col;
          *p = (ww == 0) ? dacc[u][v] : *p + dacc[u][v];
        }
      }
    }
    __syncthreads();
  }
  double* out = a.part + ((size_t)blockIdx.y * a.nblk + blockIdx.x) * RB * RB;
  for (int e = threadIdx.x; e < RB * RB; e += 256) out[e] = red[e];
}

// G from the slice partials, one wave per entry of the upper triangle:
// lane s adds slices s, s + 64, ... in order, a fixed xor butterfly adds
// the lanes, and the entry is written to both triangles.
template <int RB>
__global__ __launch_bounds__(256) void k_gram_mfma_reduce(const double* __restrict__ part, uint32_t nslice,
                                                          uint32_t nblk, uint32_t I, double* __restrict__ G,
                                                          const SampleHdr* hdr, const int32_t* st_solver) {
  if (hdr->status != 0 || *st_solver != 0) return;
  const uint32_t e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= nblk * RB * RB) return;
  const uint32_t blk = e / (RB * RB), xx = (e / RB) % RB, yy = e % RB;
  uint32_t by = 0;
  while ((by + 1) * (by + 2) / 2 <= blk) ++by;
  const uint32_t bx = blk - by * (by + 1) / 2;
  const uint32_t x = bx * RB + xx, y = by * RB + yy;
  if (x >= I || y >= I || (bx == by && xx > yy)) return;
  double acc = 0.0;
  for (uint32_t sl = lane; sl < nslice; sl += 64) acc += part[((size_t)sl * nblk + blk) * RB * RB + xx * RB + yy];
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) {
    G[(size_t)x * I + y] = acc;
    G[(size_t)y * I + x] = acc;
  }
}

template <int RB, bool Q1>
hipError_t gram_mfma_run(MfmaGramArgs a, double* G, size_t part_elems, hipStream_t st) {
  constexpr uint32_t CW = 4096 / RB;
  a.nb = (a.I + RB - 1) / RB;
  a.nblk = a.nb * (a.nb + 1) / 2;
  const uint32_t chunks = (a.J + CW - 1) / CW;
  // About 16 chunks per slice, at most 1024 workgroups' partials.
  uint32_t nslice = (chunks + 15) / 16;
  const uint32_t cap = (uint32_t)std::min<size_t>(1024 / a.nblk, part_elems / ((size_t)a.nblk * RB * RB));
  if (nslice > cap) nslice = cap;
  if (nslice < 1) nslice = 1;
  a.cps = (chunks + nslice - 1) / nslice;
  nslice = (chunks + a.cps - 1) / a.cps;
  hipLaunchKernelGGL((k_gram_mfma<RB, Q1>), dim3(a.nblk, nslice), dim3(256), 0, st, a);
  const uint32_t nent = a.nblk * RB * RB;
  hipLaunchKernelGGL((k_gram_mfma_reduce<RB>), dim3((nent + 3) / 4), dim3(256), 0, st, a.part, nslice,
                     a.nblk, a.I, G, a.hdr, a.st_solver);
  return hipGetLastError();
}

}  // namespace


bool sparse_tail_gram_ok(const ShapeInfo& si, const SolverLayout& SL, int n) {
  return SL.hosvd_kside[n] && n == si.d - 1 && si.h == si.d - 1 && si.MH <= kSparseGramMaxRows;
}

hipError_t launch_gram_tail_sparse(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                   char* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_rows_sparse, dim3((si.MH + 3) / 4), dim3(256), 0, st, si.MH, si.fMT,
                     sp.headpos, sp.coo_l, sp.rowptr, sp.coo_t, sp.colptr, sp.cscpos,
                     (double*)(ws + SL.G), sp.hdr, (const int32_t*)(ws + SL.status));
  const uint32_t nt = (si.MH + 63) / 64;
  hipLaunchKernelGGL(k_gram_mirror, dim3(nt, nt), dim3(256), 0, st, si.MH, sp.headpos,
                     (double*)(ws + SL.G), sp.hdr, (const int32_t*)(ws + SL.status));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sweep Gram of Y_(k) on MFMA (row side Y Y^T or column side Y^T Y of the
// float32 view (O, I_k, Q)), with the inputs in float32, bfloat16 or OCP
// float8 e4m3:
//   G[x][y] = sum_z M[x][z] M[y][z],  row side: M[x][z] = Y_(k)[x][z] (Z = J),
//                                     column side: M[x][z] = Y_(k)[z][x] (Z = I).
// Workgroup (block pair, slice) stages chunks of CW = 4096 / RB summation
// indices of its two RB-row blocks in LDS as float32 (coalesced along
// whichever of x, z is contiguous in Y), the next chunk's loads in flight
// while the current one is multiplied.  Each operand is converted when read
// from LDS:
//   float32  v_mfma_f32_16x16x4_f32      (4 summation indices per step)
//   bfloat16 v_mfma_f32_16x16x16_bf16    (16; round to nearest even)
//   e4m3     v_mfma_f32_16x16x32_fp8_fp8 (32; each staged RB x CW tile is
//            scaled by amax / 448, rounded to nearest even, saturating)
// Products accumulate in float32 over runs of 32 summation indices and in
// float64 across runs (times the two tiles' scales for e4m3).  Partials go to
// part[(x X + y) nslice + slice] for every x, y < X (both triangles).
// ---------------------------------------------------------------------------
struct YGramArgs {
  const float* Y;
  uint32_t I, Q, J;
  FastDiv fQ;
  int kside;
  int xfast;               // 1: consecutive x are consecutive in Y
  uint32_t X, Z;
  uint32_t nb, nblk;       // row blocks, upper-triangle block pairs
  uint32_t cps, nslice;    // chunks per slice, slices
  double* part;
  const SampleHdr* hdr;
  const int32_t* st_solver;
};

// OCP float8 e4m3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits;
// largest finite 448) of four float32 values, rounded to nearest even and
// saturated at +-448, packed into 32 bits (first value in the low byte).
// gfx950's v_cvt_pk_fp8_f32 rounds to nearest even into this format but
// does not saturate, so the values are clamped first.
__device__ __forceinline__ uint32_t to_e4m3x4(float a, float b, float c, float d) {
  auto cl = [](float x) { return fminf(fmaxf(x, -448.f), 448.f); };
  int pk = __builtin_amdgcn_cvt_pk_fp8_f32(cl(a), cl(b), 0, false);
  pk = __builtin_amdgcn_cvt_pk_fp8_f32(cl(c), cl(d), pk, true);
  return (uint32_t)pk;
}

__device__ __forceinline__ uint32_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

typedef short v4s __attribute__((ext_vector_type(4)));

template <int RB, int P>
__global__ __launch_bounds__(256) void k_gram_y_mfma(YGramArgs a) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  constexpr int CW = 4096 / RB, TB = RB / 16;
  constexpr int NT = TB * TB, TPW = NT >= 4 ? NT / 4 : 1, KSPLIT = NT >= 4 ? 1 : 4;
  constexpr int KI = P == 0 ? 4 : P == 1 ? 16 : 32;   // summation indices per MFMA
  constexpr int KS = CW / KI;
  __shared__ float Ma[RB][CW + 4];
  __shared__ float Mb[RB][CW + 4];
  __shared__ float wmax[2][4];
  uint32_t by = 0;
  while ((by + 1) * (by + 2) / 2 <= blockIdx.x) ++by;
  const uint32_t bx = blockIdx.x - by * (by + 1) / 2;
  const bool diag = bx == by;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const uint32_t nchunk = (a.Z + CW - 1) / CW;
  const uint32_t c0 = blockIdx.y * a.cps;
  const uint32_t c1 = min(nchunk, c0 + a.cps);
  // element u of this thread in a staged tile: (x, z) within the tile
  auto xz = [&](int u, int& x, int& z) {
    const int e = threadIdx.x + 256 * u;
    if (a.xfast) {
      x = e % RB;
      z = e / RB;
    } else {
      z = e % CW;
      x = e / CW;
    }
  };
  auto load = [&](uint32_t row0, uint32_t zc, float* v) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      int x, z;
      xz(u, x, z);
      const uint32_t xg = row0 + x, zg = zc + z;
      float val = 0.f;
      if (xg < a.X && zg < a.Z) {
        const uint32_t j = a.kside ? xg : zg, i = a.kside ? zg : xg;
        const uint32_t q = a.fQ.div(j);
        val = a.Y[(size_t)q * a.I * a.Q + (j - q * a.Q) + (size_t)i * a.Q];
      }
      v[u] = val;
    }
  };
  v4f acc[TPW];
  double dacc[TPW][4];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) dacc[u][v] = 0.0;
  }
  float va[16], vb[16];
  if (c0 < c1) {
    load(bx * RB, c0 * CW, va);
    if (!diag) load(by * RB, c0 * CW, vb);
  }
  for (uint32_t c = c0; c < c1; ++c) {
    __syncthreads();
    float ma = 0.f, mb = 0.f;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      int x, z;
      xz(u, x, z);
      Ma[x][z] = va[u];
      ma = fmaxf(ma, fabsf(va[u]));
      if (!diag) {
        Mb[x][z] = vb[u];
        mb = fmaxf(mb, fabsf(vb[u]));
      }
    }
    if constexpr (P == 2) {
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) {
        ma = fmaxf(ma, __shfl_xor(ma, m, 64));
        mb = fmaxf(mb, __shfl_xor(mb, m, 64));
      }
      if (lane == 0) {
        wmax[0][w] = ma;
        wmax[1][w] = mb;
      }
    }
    __syncthreads();
    if (c + 1 < c1) {
      load(bx * RB, (c + 1) * CW, va);
      if (!diag) load(by * RB, (c + 1) * CW, vb);
    }
    float sa = 1.f, sb = 1.f;
    if constexpr (P == 2) {
      const float amax = fmaxf(fmaxf(wmax[0][0], wmax[0][1]), fmaxf(wmax[0][2], wmax[0][3]));
      const float bmax = diag ? amax : fmaxf(fmaxf(wmax[1][0], wmax[1][1]), fmaxf(wmax[1][2], wmax[1][3]));
      sa = amax > 0.f ? amax / 448.f : 1.f;
      sb = bmax > 0.f ? bmax / 448.f : 1.f;
    }
    const float ia = 1.f / sa, ib = 1.f / sb;
    const double sab = (double)sa * (double)sb;
    float (*B)[CW + 4] = diag ? Ma : Mb;
    // float32 runs of 32 summation indices, then float64 (as for a scalar
    // Gram: the float32 rounding of a run stays at about 32 u)
    constexpr int FLUSH = KI >= 32 ? 1 : 32 / KI;
    int run = 0;
    for (int ks = (KSPLIT > 1 ? w : 0); ks < KS; ks += KSPLIT) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int t = (NT >= 4 ? w * TPW : 0) + u, x = t / TB, y = t % TB;
        const float* ra = &Ma[x * 16 + li][ks * KI];
        const float* rb = &B[y * 16 + li][ks * KI];
        if constexpr (P == 0) {
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[lk], rb[lk], acc[u], 0, 0, 0);
        } else if constexpr (P == 1) {
          v4s oa, ob;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            oa[q] = (short)to_bf16(ra[4 * lk + q]);
            ob[q] = (short)to_bf16(rb[4 * lk + q]);
          }
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(oa, ob, acc[u], 0, 0, 0);
        } else {
          const float* pa = ra + 8 * lk;
          const float* pb = rb + 8 * lk;
          const uint64_t oa = (uint64_t)to_e4m3x4(pa[0] * ia, pa[1] * ia, pa[2] * ia, pa[3] * ia) |
                              ((uint64_t)to_e4m3x4(pa[4] * ia, pa[5] * ia, pa[6] * ia, pa[7] * ia) << 32);
          const uint64_t ob = (uint64_t)to_e4m3x4(pb[0] * ib, pb[1] * ib, pb[2] * ib, pb[3] * ib) |
                              ((uint64_t)to_e4m3x4(pb[4] * ib, pb[5] * ib, pb[6] * ib, pb[7] * ib) << 32);
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)oa, (long)ob, acc[u], 0, 0, 0);
        }
      }
      if (++run == FLUSH) {
        run = 0;
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
#pragma unroll
          for (int v = 0; v < 4; ++v) dacc[u][v] += (double)acc[u][v] * sab;
          acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[u][v] += (double)acc[u][v] * sab;
      acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  __syncthreads();
  double* red = reinterpret_cast<double*>(&Ma[0][0]);
  static_assert(sizeof(Ma) + sizeof(Mb) >= RB * RB * sizeof(double), "reduction buffer");
  for (int ww = 0; ww < KSPLIT; ++ww) {
    if (KSPLIT == 1 || w == ww) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int t = (NT >= 4 ? w * TPW : 0) + u, x = t / TB, y = t % TB;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* p = red + (x * 16 + lk * 4 + v) * RB + (y * 16 + li);
          *p = (ww == 0) ? dacc[u][v] : *p + dacc[u][v];
        }
      }
    }
    __syncthreads();
  }
  const uint32_t sl = blockIdx.y;
  for (int e = threadIdx.x; e < RB * RB; e += 256) {
    const uint32_t xx = e / RB, yy = e % RB, x = bx * RB + xx, y = by * RB + yy;
    if (x >= a.X || y >= a.X) continue;
    a.part[((size_t)x * a.X + y) * a.nslice + sl] = red[e];
    if (!diag) a.part[((size_t)y * a.X + x) * a.nslice + sl] = red[e];
  }
}

template <int RB, int P>
hipError_t gram_y_mfma_go(YGramArgs a, hipStream_t st) {
  hipLaunchKernelGGL((k_gram_y_mfma<RB, P>), dim3(a.nblk, a.nslice), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int P>
hipError_t gram_y_mfma_rb(const YGramArgs& a, int rb, hipStream_t st) {
  if (rb == 16) return gram_y_mfma_go<16, P>(a, st);
  if (rb == 32) return gram_y_mfma_go<32, P>(a, st);
  return gram_y_mfma_go<64, P>(a, st);
}

// Sets up and launches the MFMA sweep Gram of Y_k into SL.Gpart; returns
// the number of slices in *nslice.  prec: MACH_F32, MACH_BF16 or
// MACH_FP8E4M3 (the Gram's input precision).
hipError_t gram_y_mfma(const SolverLayout& SL, char* ws, int k, int prec, const SampleHdr* hdr,
                       hipStream_t st, uint32_t* nslice) {
  const ModePlan& m = SL.mp[k];
  YGramArgs a{};
  a.Y = (const float*)(ws + m.ybuf);
  a.I = m.I;
  a.Q = m.Q;
  a.J = m.O * m.Q;
  a.fQ = make_fastdiv(m.Q);
  a.kside = m.kside;
  a.xfast = m.kside ? (m.Q > 1) : (m.Q == 1);
  a.X = m.s;
  a.Z = m.kside ? m.I : a.J;
  a.part = (double*)(ws + SL.Gpart);
  a.hdr = hdr;
  a.st_solver = (const int32_t*)(ws + SL.status);
  const int rb = a.X <= 16 ? 16 : a.X <= 32 ? 32 : 64;
  const uint32_t cw = 4096u / (uint32_t)rb;
  a.nb = (a.X + rb - 1) / rb;
  a.nblk = a.nb * (a.nb + 1) / 2;
  const uint32_t chunks = (a.Z + cw - 1) / cw;
  // Slices of at least 4 chunks, at most 256, enough workgroups to fill
  // the chip when there are chunks for it, and partials that fit Gpart.
  const uint64_t n2 = (uint64_t)a.X * a.X;
  uint32_t ns = 1;
  while (ns < 256 && (uint64_t)a.nblk * ns < 512 && chunks >= 8u * ns && n2 * 2 * ns <= SL.Gpart_elems) ns *= 2;
  a.cps = (chunks + ns - 1) / ns;
  a.nslice = (chunks + a.cps - 1) / a.cps;
  *nslice = a.nslice;
  if (prec == MACH_BF16) return gram_y_mfma_rb<1>(a, rb, st);
  if (prec == MACH_FP8E4M3) return gram_y_mfma_rb<2>(a, rb, st);
  return gram_y_mfma_rb<0>(a, rb, st);
}

// Gram partials of Y_k: SL.Gpart[X][X][c], c < *nchunk.
hipError_t launch_gram_y_partials(const SolverLayout& SL, char* ws, int k, int prec,
                                  const SampleHdr* hdr, hipStream_t st, uint32_t* nchunk) {
  return gram_y_mfma(SL, ws, k, prec, hdr, st, nchunk);
}

// Gram of Y_k into SL.G.
hipError_t launch_gram_y(const SolverLayout& SL, char* ws, int k, int prec, const SampleHdr* hdr,
                         hipStream_t st) {
  uint32_t ns = 1;
  hipError_t e = gram_y_mfma(SL, ws, k, prec, hdr, st, &ns);
  if (e != hipSuccess) return e;
  const uint32_t n2 = SL.mp[k].s * SL.mp[k].s;
  hipLaunchKernelGGL(k_gram_reduce, dim3((n2 + 255) / 256), dim3(256), 0, st,
                     (const double*)(ws + SL.Gpart), ns, n2, (double*)(ws + SL.G), hdr,
                     (const int32_t*)(ws + SL.status));
  return hipGetLastError();
}

// Gram of the sampled unfolding Xhat_(n) (unscaled values) into SL.G.
hipError_t launch_gram_xhat(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                            char* ws, int n, hipStream_t st) {
  GramArgs a{};
  a.I = si.dims[n];
  a.Q = si.stride[n];
  a.J = si.N / si.dims[n];
  a.fQ = si.fstride[n];
  a.kside = SL.hosvd_kside[n];
  a.X = SL.hosvd_s[n];
  a.Z = a.kside ? a.I : a.J;
  a.part = (double*)(ws + SL.Gpart);
  a.st_solver = (const int32_t*)(ws + SL.status);
  a.hdr = sp.hdr;
  const bool q1 = a.Q == 1 && a.I % 64 == 0;   // the last mode, 64-aligned
  if (!a.kside && (a.Q % 64 == 0 || q1) && a.I <= kMfmaGramMaxRows) {
    MfmaGramArgs m{};
    m.bitmap = sp.bitmap;
    m.wrank = sp.wrank;
    m.coo = sp.coo_l;
    m.I = a.I;
    m.Q = a.Q;
    m.J = a.J;
    m.fQ = a.fQ;
    m.part = a.part;
    m.hdr = sp.hdr;
    m.st_solver = a.st_solver;
    double* G = (double*)(ws + SL.G);
    if (q1) return gram_mfma_run<64, true>(m, G, SL.Gpart_elems, st);
    if (a.I <= 16) return gram_mfma_run<16, false>(m, G, SL.Gpart_elems, st);
    if (a.I <= 32) return gram_mfma_run<32, false>(m, G, SL.Gpart_elems, st);
    return gram_mfma_run<64, false>(m, G, SL.Gpart_elems, st);
  }
  MaskedLoad ld{sp.bitmap, sp.wrank, sp.coo_l};
  return gram_run(a, ld, (double*)(ws + SL.G), SL.Gpart_elems, st);
}

}  // namespace mach
