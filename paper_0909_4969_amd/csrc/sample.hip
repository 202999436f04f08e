// MACH coin toss (Alg. 1/2, "MACH" block; Theorem 1; Remark 1) and the
// sparse layouts built from it.
//
// Pipeline (all on one stream, no host synchronisation):
//   init      header fields (p, threshold, capacity, seed, window)
//   mask      Philox4x32-10 word per linear index -> keep bitmap, one 64-bit
//             word per thread, and a kept count per 16384-entry block
//   scan      exclusive scan of the block counts (one workgroup)
//   compact   per block: word ranks, then every kept entry written as
//             (l, float32 x_l) at its rank, plus sum x^2 in float64
//   finalize  kept count, sum x^2 (fixed-order tree), capacity status
//   rowptr    CSR row pointers = rank of each head row's first index
//   headrow   head row index of each position in the CSC head order
//   csc_count / scan / csc_fill   the CSC copy: for every tail column c,
//             its kept entries ordered by the head coordinates in headperm
//             order.  A column is read by 64 lanes at once (64 consecutive c
//             share bitmap words), so no sort is needed.
#include <cmath>

#include "mach_internal.h"

namespace mach {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-wide sum over 256 threads in a fixed order; result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum256(T v, T* sh) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// Exclusive scan over 256 threads; returns the exclusive prefix, total in *tot.
__device__ __forceinline__ uint32_t block_exscan256(uint32_t v, uint32_t* sh, uint32_t* tot) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int i = 0; i < w; ++i) base += sh[i];
  *tot = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return base + x - v;
}

__global__ void k_sample_init(SampleHdr* hdr, double p, uint64_t thresh, uint64_t cap,
                              uint64_t seed, uint64_t window, uint64_t coin) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hdr->coin = coin;
    hdr->nnz = 0;
    hdr->cap = cap;
    hdr->p = p;
    hdr->sumsq = 0.0;
    hdr->thresh = thresh;
    hdr->seed = seed;
    hdr->window = window;
    hdr->status = 0;
    hdr->magic = kSampleMagic;
  }
}

// One thread per 64-bit bitmap word: 16 Philox blocks, 4 words each.
__global__ __launch_bounds__(kThreads) void k_sample_mask(uint32_t N, uint64_t thresh, uint32_t s_lo,
                                                          uint32_t s_hi, uint32_t w_lo, uint32_t w_hi,
                                                          uint64_t* __restrict__ bitmap,
                                                          uint32_t* __restrict__ blkcnt) {
  __shared__ uint32_t sh[4];
  uint32_t w = blockIdx.x * kSampleBlockWords + threadIdx.x;
  uint64_t bits = 0;
  uint32_t l0 = w * 64u;
  if (l0 < N) {
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      uint32_t c[4] = {w * 16u + (uint32_t)j, 0u, w_lo, w_hi};
      philox4x32_10(c, s_lo, s_hi);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint32_t l = l0 + 4u * j + k;
        uint64_t keep = ((uint64_t)c[k] < thresh) && (l < N);
        bits |= keep << (4 * j + k);
      }
    }
  }
  bitmap[w] = bits;
  uint32_t tot = block_sum256<uint32_t>((uint32_t)__popcll(bits), sh);
  if (threadIdx.x == 0) blkcnt[blockIdx.x] = tot;
}

// Tick-keyed coins for a window of consecutive ticks of a stream: the last
// mode is time, entry l = j T + t (j the series, the flat index of the other
// coordinates; t the tick within the window) gets word tau mod 4 of the
// Philox block at counter (q lo, q hi, j, 0), q = tau / 4, tau = tick0 + t,
// key (seed lo, seed hi).  A measurement gets the same coin in every window
// that contains it.  One thread per 64-bit bitmap word; a block is computed
// once for the (up to four) consecutive ticks that share it.
__global__ __launch_bounds__(kThreads) void k_sample_mask_ticks(uint32_t N, FastDiv fT, uint64_t thresh,
                                                                uint32_t s_lo, uint32_t s_hi,
                                                                uint64_t tick0,
                                                                uint64_t* __restrict__ bitmap,
                                                                uint32_t* __restrict__ blkcnt) {
  __shared__ uint32_t sh[4];
  const uint32_t w = blockIdx.x * kSampleBlockWords + threadIdx.x;
  uint64_t bits = 0;
  const uint32_t l0 = w * 64u;
  if (l0 < N) {
    uint32_t j = fT.div(l0), t = l0 - j * fT.d;
    uint64_t tau = tick0 + t;
    uint32_t c[4] = {0u, 0u, 0u, 0u};
    uint64_t cq = ~0ull;
    uint32_t cj = ~0u;
    const uint32_t nb = min(64u, N - l0);
    for (uint32_t b = 0; b < nb; ++b) {
      const uint64_t q = tau >> 2;
      if (q != cq || j != cj) {
        c[0] = (uint32_t)q;
        c[1] = (uint32_t)(q >> 32);
        c[2] = j;
        c[3] = 0u;
        philox4x32_10(c, s_lo, s_hi);
        cq = q;
        cj = j;
      }
      const uint32_t sel = (uint32_t)tau & 3u;
      const uint32_t word = sel == 0 ? c[0] : sel == 1 ? c[1] : sel == 2 ? c[2] : c[3];
      bits |= (uint64_t)((uint64_t)word < thresh) << b;
      if (++t == fT.d) {
        t = 0;
        ++j;
        tau = tick0;
      } else {
        ++tau;
      }
    }
  }
  bitmap[w] = bits;
  uint32_t tot = block_sum256<uint32_t>((uint32_t)__popcll(bits), sh);
  if (threadIdx.x == 0) blkcnt[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// Sliding window of a stream (Remark 2: a coin per measurement as it
// arrives): the window of ticks tick0 .. tick0 + T - 1 built from the sample
// of an earlier window of the same series (ticks tick0p .. tick0p + T - 1,
// same seed, keep threshold and capacity).  A measurement (j, tau) inside
// the earlier window keeps that window's coin and kept value (its bit and
// its entry are copied, no Philox block and no read of X); a measurement
// outside it is tossed as in k_sample_mask_ticks and its value read from X.
// Coins are keyed on (seed, j, tau) either way, so the result equals a fresh
// toss of the whole window bit for bit.  If the earlier sample is not a
// valid tick-keyed sample with the same seed, threshold and capacity, every
// measurement is tossed afresh.
// ---------------------------------------------------------------------------
struct PrevSample {
  const SampleHdr* hdr;
  const uint64_t* bitmap;
  const uint32_t* wrank;
  const Entry* coo;
};

// Kept entries with linear index below l (reads no bitmap word past the
// last one when l is a multiple of 64).
__device__ __forceinline__ uint32_t rank_at(const uint64_t* bitmap, const uint32_t* wrank, uint32_t l) {
  return (l & 63u) ? bit_rank(bitmap, wrank, l) : wrank[l >> 6];
}

__device__ __forceinline__ bool prev_usable(const PrevSample& pv, uint64_t seed, uint64_t thresh,
                                            uint64_t cap) {
  const SampleHdr* h = pv.hdr;
  return h->magic == kSampleMagic && h->coin == 1 && h->seed == seed && h->thresh == thresh &&
         h->cap == cap && h->status == 0 && h->nnz <= cap;
}

__global__ __launch_bounds__(kThreads) void k_sample_mask_slide(uint32_t N, FastDiv fT, uint64_t thresh,
                                                                uint64_t seed, uint64_t tick0,
                                                                uint64_t cap, PrevSample pv,
                                                                uint64_t* __restrict__ bitmap,
                                                                uint32_t* __restrict__ blkcnt) {
  __shared__ uint32_t sh[4];
  const uint32_t s_lo = (uint32_t)seed, s_hi = (uint32_t)(seed >> 32);
  const bool reuse = prev_usable(pv, seed, thresh, cap);
  const uint64_t tick0p = pv.hdr->window;
  const uint32_t w = blockIdx.x * kSampleBlockWords + threadIdx.x;
  uint64_t bits = 0;
  const uint32_t l0 = w * 64u;
  if (l0 < N) {
    uint32_t j = fT.div(l0), t = l0 - j * fT.d;
    uint64_t tau = tick0 + t;
    uint32_t c[4] = {0u, 0u, 0u, 0u};
    uint64_t cq = ~0ull;
    uint32_t cj = ~0u;
    uint32_t pw = ~0u;
    uint64_t pword = 0;
    const uint32_t nb = min(64u, N - l0);
    for (uint32_t b = 0; b < nb; ++b) {
      const uint64_t tp = tau - tick0p;      // position in the earlier window (wraps if before it)
      uint64_t keep;
      if (reuse && tp < fT.d) {
        const uint32_t lp = j * fT.d + (uint32_t)tp;
        if ((lp >> 6) != pw) {
          pw = lp >> 6;
          pword = pv.bitmap[pw];
        }
        keep = (pword >> (lp & 63u)) & 1ull;
      } else {
        const uint64_t q = tau >> 2;
        if (q != cq || j != cj) {
          c[0] = (uint32_t)q;
          c[1] = (uint32_t)(q >> 32);
          c[2] = j;
          c[3] = 0u;
          philox4x32_10(c, s_lo, s_hi);
          cq = q;
          cj = j;
        }
        const uint32_t sel = (uint32_t)tau & 3u;
        const uint32_t word = sel == 0 ? c[0] : sel == 1 ? c[1] : sel == 2 ? c[2] : c[3];
        keep = (uint64_t)word < thresh;
      }
      bits |= keep << b;
      if (++t == fT.d) {
        t = 0;
        ++j;
        tau = tick0;
      } else {
        ++tau;
      }
    }
  }
  bitmap[w] = bits;
  uint32_t tot = block_sum256<uint32_t>((uint32_t)__popcll(bits), sh);
  if (threadIdx.x == 0) blkcnt[blockIdx.x] = tot;
}

// Single-workgroup exclusive scan in place over a[0..n); a[n] receives the total.
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* __restrict__ a, uint32_t n) {
  __shared__ uint32_t part[1024];
  uint32_t t = threadIdx.x;
  uint32_t chunk = (n + 1023) / 1024;
  uint32_t b = t * chunk, e = min(n, b + chunk);
  uint32_t s = 0;
  for (uint32_t i = b; i < e; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over 1024 partials.
  for (uint32_t o = 1; o < 1024; o <<= 1) {
    uint32_t y = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  uint32_t run = part[t] - s;
  for (uint32_t i = b; i < e; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  if (t == 1023) a[n] = part[1023];
}

// Multi-block exclusive scan in place over a[0..n) with a[n] = total:
// per-block sums, one-workgroup scan of those, then per-block rescan.
constexpr uint32_t kScanBlock = 4096;

__global__ __launch_bounds__(256) void k_scan_blocksum(const uint32_t* __restrict__ a, uint32_t n,
                                                       uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[4];
  uint32_t b0 = blockIdx.x * kScanBlock, s = 0;
  for (uint32_t i = b0 + threadIdx.x; i < min(n, b0 + kScanBlock); i += 256) s += a[i];
  s = block_sum256<uint32_t>(s, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t* __restrict__ a, uint32_t n,
                                                    const uint32_t* __restrict__ boff) {
  __shared__ uint32_t sh[4];
  const uint32_t b0 = blockIdx.x * kScanBlock;
  uint32_t run = boff[blockIdx.x];
  // 16 elements per thread, contiguous per thread
  const uint32_t base = b0 + threadIdx.x * 16;
  uint32_t v[16], s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = (base + k < n) ? a[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exscan256(s, sh, &tot);
  run += ex;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (base + k < n) a[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) a[n] = boff[gridDim.x];
}

void scan_u32(uint32_t* a, uint32_t n, uint32_t* bsum, hipStream_t st) {
  uint32_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, a, n);
    return;
  }
  hipLaunchKernelGGL(k_scan_blocksum, dim3(nb), dim3(256), 0, st, a, n, bsum);
  hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, bsum, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, st, a, n, bsum);
}

// Four consecutive inputs at a 4-element-aligned index (the tensor base is
// at least 16-byte aligned): one 16-byte load for float, two for double.
__device__ __forceinline__ void load4(const float* p, float x[4]) {
  float4 v = *reinterpret_cast<const float4*>(p);
  x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double x[4]) {
  double2 a = reinterpret_cast<const double2*>(p)[0];
  double2 b = reinterpret_cast<const double2*>(p)[1];
  x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
}

template <typename XT>
__global__ __launch_bounds__(kThreads) void k_sample_compact(const XT* __restrict__ X, uint32_t N,
                                                             const uint64_t* __restrict__ bitmap,
                                                             const uint32_t* __restrict__ blkoff,
                                                             uint32_t* __restrict__ wrank,
                                                             Entry* __restrict__ coo, uint64_t cap,
                                                             double* __restrict__ sumsq_part) {
  __shared__ uint64_t words[kSampleBlockWords];
  __shared__ uint32_t lrank[kSampleBlockWords];
  __shared__ uint32_t sh[4];
  __shared__ double shd[4];
  const uint32_t b = blockIdx.x;
  const uint32_t base_word = b * kSampleBlockWords;
  const uint64_t myword = bitmap[base_word + threadIdx.x];
  uint32_t tot;
  uint32_t ex = block_exscan256((uint32_t)__popcll(myword), sh, &tot);
  const uint32_t off = blkoff[b];
  wrank[base_word + threadIdx.x] = off + ex;
  words[threadIdx.x] = myword;
  lrank[threadIdx.x] = ex;
  __syncthreads();
  double ss = 0.0;
  const uint32_t base_elem = b * kSampleBlockElems;
  // The X loads of all 16 groups of four elements (those with a kept entry)
  // are issued before any entry is written.
  XT xs[16][4];
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const uint32_t g = it * kThreads + threadIdx.x;
    const uint32_t e0 = base_elem + 4u * g;
    const uint32_t nib = (uint32_t)(words[g >> 4] >> ((g & 15u) * 4u)) & 15u;
    if (nib != 0) {
      if (e0 + 3 < N) {
        load4(X + e0, xs[it]);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) xs[it][k] = (e0 + k < N) ? X[e0 + k] : (XT)0;
      }
    }
  }
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    uint32_t g = it * kThreads + threadIdx.x;
    uint32_t e0 = base_elem + 4u * g;
    uint32_t wi = g >> 4, sh4 = (g & 15u) * 4u;
    uint64_t word = words[wi];
    uint32_t nib = (uint32_t)(word >> sh4) & 15u;
    if (nib == 0) continue;
    uint64_t below = sh4 ? (word & ((~0ull) >> (64 - sh4))) : 0ull;
    uint64_t r = (uint64_t)off + lrank[wi] + (uint32_t)__popcll(below);
    const XT* x = xs[it];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if ((nib >> k) & 1u) {
        double xv = (double)x[k];
        if (r < cap) {
          Entry en;
          en.l = e0 + k;
          en.v = (float)x[k];
          coo[r] = en;
        }
        ss += xv * xv;
        ++r;
      }
    }
  }
  double s = block_sum256<double>(ss, shd);
  if (threadIdx.x == 0) sumsq_part[b] = s;
}

// Word ranks of a block (as the prologue of k_sample_compact).
__global__ __launch_bounds__(kThreads) void k_word_ranks(const uint64_t* __restrict__ bitmap,
                                                         const uint32_t* __restrict__ blkoff,
                                                         uint32_t* __restrict__ wrank) {
  __shared__ uint32_t sh[4];
  const uint32_t w = blockIdx.x * kSampleBlockWords + threadIdx.x;
  uint32_t tot;
  const uint32_t ex = block_exscan256((uint32_t)__popcll(bitmap[w]), sh, &tot);
  wrank[w] = blkoff[blockIdx.x] + ex;
}

// The shared measurements of a slid window, one wave per series j: in both
// windows they are one run of the l-ordered kept list (ticks a .. b - 1 of
// the new window, a + shift .. b + shift - 1 of the earlier one, shift =
// tick0 - tick0p), so the run is copied with its linear indices moved by
// -shift.  Nothing is copied when the earlier sample is not usable.
__global__ __launch_bounds__(256) void k_slide_copy_runs(uint32_t nseries, uint32_t T, uint64_t tick0,
                                                         uint64_t seed, uint64_t thresh, uint64_t cap,
                                                         PrevSample pv,
                                                         const uint64_t* __restrict__ bitmap,
                                                         const uint32_t* __restrict__ wrank,
                                                         const uint32_t* __restrict__ total,
                                                         Entry* __restrict__ coo) {
  if (!prev_usable(pv, seed, thresh, cap)) return;
  const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= nseries) return;
  const uint64_t tick0p = pv.hdr->window;
  // overlap in new-window ticks [a, b)
  const int64_t shift = (int64_t)(tick0 - tick0p);   // ticks wrap to a signed difference
  const int64_t a64 = shift < 0 ? -shift : 0, b64 = shift < 0 ? (int64_t)T : (int64_t)T - shift;
  if (a64 >= b64 || a64 >= (int64_t)T) return;
  const uint32_t a = (uint32_t)a64, b = (uint32_t)b64;
  // ranks in the new window (its word ranks are written, its total is the
  // scan's last entry: wrank past the last word is not written yet)
  const uint32_t N = nseries * T;
  const uint32_t dst0 = rank_at(bitmap, wrank, j * T + a);
  const uint32_t dst1 = j * T + b == N ? *total : rank_at(bitmap, wrank, j * T + b);
  const uint32_t src0 = rank_at(pv.bitmap, pv.wrank, (uint32_t)((int64_t)(j * T + a) + shift));
  const uint32_t n = dst1 - dst0;
  for (uint32_t k = lane; k < n; k += 64) {
    Entry e = pv.coo[src0 + k];
    e.l = (uint32_t)((int64_t)e.l - shift);
    if (dst0 + k < cap) coo[dst0 + k] = e;
  }
}

// Compaction of a slid window: as k_sample_compact (same elements per
// thread, same order, so the same sum of squares), the values of the shared
// measurements read back from the kept list where k_slide_copy_runs put
// them, the others from X and written.
template <typename XT>
__global__ __launch_bounds__(kThreads) void k_sample_compact_slide(const XT* __restrict__ X, uint32_t N,
                                                                   FastDiv fT, uint64_t tick0,
                                                                   uint64_t seed, uint64_t thresh,
                                                                   PrevSample pv,
                                                                   const uint64_t* __restrict__ bitmap,
                                                                   const uint32_t* __restrict__ blkoff,
                                                                   const uint32_t* __restrict__ wrank,
                                                                   Entry* __restrict__ coo, uint64_t cap,
                                                                   double* __restrict__ sumsq_part) {
  __shared__ uint64_t words[kSampleBlockWords];
  __shared__ uint32_t lrank[kSampleBlockWords];
  __shared__ double shd[4];
  // float64 input: the sum of squares needs the float64 value, which the
  // earlier sample does not hold, so only its coins are reused
  const bool reuse = sizeof(XT) == 4 && prev_usable(pv, seed, thresh, cap);
  const uint64_t tick0p = pv.hdr->window;
  const uint32_t b = blockIdx.x;
  const uint32_t base_word = b * kSampleBlockWords;
  const uint32_t off = blkoff[b];
  words[threadIdx.x] = bitmap[base_word + threadIdx.x];
  lrank[threadIdx.x] = wrank[base_word + threadIdx.x] - off;
  __syncthreads();
  double ss = 0.0;
  const uint32_t base_elem = b * kSampleBlockElems;
  for (int it = 0; it < 16; ++it) {
    uint32_t g = it * kThreads + threadIdx.x;
    uint32_t e0 = base_elem + 4u * g;
    uint32_t wi = g >> 4, sh4 = (g & 15u) * 4u;
    uint64_t word = words[wi];
    uint32_t nib = (uint32_t)(word >> sh4) & 15u;
    if (nib == 0) continue;
    uint64_t below = sh4 ? (word & ((~0ull) >> (64 - sh4))) : 0ull;
    uint64_t r = (uint64_t)off + lrank[wi] + (uint32_t)__popcll(below);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if ((nib >> k) & 1u) {
        const uint32_t l = e0 + k;
        const uint64_t tp = tick0 + fT.mod(l) - tick0p;   // tick in the earlier window
        double xv;
        if (reuse && tp < fT.d) {
          xv = (double)(r < cap ? coo[r].v : 0.f);
        } else {
          const XT x = X[l];
          xv = (double)x;
          if (r < cap) {
            Entry en;
            en.l = l;
            en.v = (float)x;
            coo[r] = en;
          }
        }
        ss += xv * xv;
        ++r;
      }
    }
  }
  double s = block_sum256<double>(ss, shd);
  if (threadIdx.x == 0) sumsq_part[b] = s;
}

__global__ __launch_bounds__(256) void k_sample_finalize(SampleHdr* hdr, const uint32_t* blkoff,
                                                         uint32_t nblk, const double* sumsq_part,
                                                         uint32_t* wrank, uint32_t nwords) {
  __shared__ double shd[4];
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < nblk; i += 256) s += sumsq_part[i];
  s = block_sum256<double>(s, shd);
  if (threadIdx.x == 0) {
    uint64_t nnz = blkoff[nblk];
    hdr->nnz = nnz;
    hdr->sumsq = s;
    wrank[nwords] = (uint32_t)nnz;
    // No kept value other than zero: every Gram of the sampled tensor is
    // zero and no subspace is determined.  A kept value that is not finite
    // would poison every product.  Either way the solver calls that follow
    // on this sample do nothing (their kernels check this status).
    if (nnz > hdr->cap) hdr->status = MACH_ENOMEM;
    else if (!(s < INFINITY)) hdr->status = MACH_EINVAL;
    else if (s == 0.0) hdr->status = MACH_EDEGENERATE;
  }
}

__global__ void k_rowptr(ShapeInfo si, const uint64_t* __restrict__ bitmap,
                         const uint32_t* __restrict__ wrank, const SampleHdr* hdr,
                         uint32_t* __restrict__ rowptr) {
  uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > si.MH) return;
  uint64_t cap = hdr->cap;
  uint64_t v = (r == si.MH) ? hdr->nnz : (uint64_t)bit_rank(bitmap, wrank, r * si.MT);
  rowptr[r] = (uint32_t)(v < cap ? v : cap);
}

// headrow[t] = C-order head row index of position t in headperm order.
__global__ void k_headrow(ShapeInfo si, uint32_t* __restrict__ headrow, uint32_t* __restrict__ headpos) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= si.MH) return;
  uint32_t rem = t, r = 0;
  for (int j = si.h - 1; j >= 0; --j) {
    int m = si.headperm[j];
    uint32_t i = si.fdim[m].mod(rem);
    rem = si.fdim[m].div(rem);
    r += i * (si.stride[m] / si.MT);
  }
  headrow[t] = r;
  headpos[r] = t;
}

// Wave = (64 consecutive tail columns) x (one block of rb head rows).
constexpr int kCscRows = 8;   // rows of a CSC count / fill group

__global__ __launch_bounds__(256) void k_csc_count(ShapeInfo si, const uint64_t* __restrict__ bitmap,
                                                   const uint32_t* __restrict__ headrow,
                                                   uint32_t* __restrict__ cnt) {
  uint32_t rb = blockIdx.y * 4 + (threadIdx.x >> 6);
  uint32_t c = blockIdx.x * 64 + (threadIdx.x & 63);
  if (rb >= si.nrb || c >= si.MT) return;
  uint32_t t0 = rb * si.rb, t1 = min(si.MH, t0 + si.rb);
  uint32_t n = 0;
  // rows in groups of kCscRows, their loads issued before any is used
  // (indices clamped to the block's last row; the extra rows are not counted)
  for (uint32_t tb = t0; tb < t1; tb += kCscRows) {
    uint64_t word[kCscRows];
    uint32_t l[kCscRows];
#pragma unroll
    for (int u = 0; u < kCscRows; ++u) {
      l[u] = headrow[min(tb + u, t1 - 1)] * si.MT + c;
      word[u] = bitmap[l[u] >> 6];
    }
#pragma unroll
    for (int u = 0; u < kCscRows; ++u)
      n += tb + u < t1 ? (uint32_t)(word[u] >> (l[u] & 63)) & 1u : 0u;
  }
  cnt[c * si.nrb + rb] = n;
}

__global__ __launch_bounds__(256) void k_csc_fill(ShapeInfo si, const uint64_t* __restrict__ bitmap,
                                                  const uint32_t* __restrict__ wrank,
                                                  const uint32_t* __restrict__ headrow,
                                                  const uint32_t* __restrict__ cnt,
                                                  const Entry* __restrict__ coo_l,
                                                  Entry* __restrict__ coo_t, uint32_t* __restrict__ colptr,
                                                  uint32_t* __restrict__ cscpos, const SampleHdr* hdr) {
  uint32_t rb = blockIdx.y * 4 + (threadIdx.x >> 6);
  uint32_t c = blockIdx.x * 64 + (threadIdx.x & 63);
  if (rb >= si.nrb || c >= si.MT) return;
  const uint64_t cap = hdr->cap;
  uint64_t dest = cnt[c * si.nrb + rb];
  if (rb == 0) colptr[c] = (uint32_t)(dest < cap ? dest : cap);
  if (rb == 0 && c == 0) {
    uint64_t nnz = hdr->nnz;
    colptr[si.MT] = (uint32_t)(nnz < cap ? nnz : cap);
  }
  if (cap == 0) return;
  uint32_t t0 = rb * si.rb, t1 = min(si.MH, t0 + si.rb);
  // Rows in groups of kCscRows: the bitmap words and word ranks of the group,
  // then its entries, are loaded before any is used (indices clamped to the
  // block's last row and to the kept list; the extra loads are not used), and
  // the kept entries are placed in row order as before.
  for (uint32_t tb = t0; tb < t1; tb += kCscRows) {
    uint64_t word[kCscRows], src[kCscRows];
    uint32_t l[kCscRows], wr[kCscRows];
    Entry en[kCscRows];
#pragma unroll
    for (int u = 0; u < kCscRows; ++u) {
      l[u] = headrow[min(tb + u, t1 - 1)] * si.MT + c;
      word[u] = bitmap[l[u] >> 6];
      wr[u] = wrank[l[u] >> 6];
    }
#pragma unroll
    for (int u = 0; u < kCscRows; ++u) {
      const uint32_t b = l[u] & 63;
      const uint64_t below = b ? (word[u] & ((~0ull) >> (64 - b))) : 0ull;
      src[u] = (uint64_t)wr[u] + (uint32_t)__popcll(below);
      en[u] = coo_l[src[u] < cap ? src[u] : cap - 1];
    }
#pragma unroll
    for (int u = 0; u < kCscRows; ++u) {
      if (tb + u < t1 && ((word[u] >> (l[u] & 63)) & 1ull)) {
        if (src[u] < cap && dest < cap) {
          coo_t[dest] = en[u];
          cscpos[src[u]] = (uint32_t)dest;
        }
        ++dest;
      }
    }
  }
}

}  // namespace

hipError_t launch_sample(const ShapeInfo& si, int x_is_f64, const void* X, double p, uint64_t seed,
                         uint64_t window, char* ws, const SampleLayout& L, uint64_t cap,
                         hipStream_t st, int coin) {
  SampleHdr* hdr = (SampleHdr*)(ws + L.hdr);
  uint64_t* bitmap = (uint64_t*)(ws + L.bitmap);
  uint32_t* wrank = (uint32_t*)(ws + L.wrank);
  uint32_t* blkcnt = (uint32_t*)(ws + L.blkcnt);
  double* sumsq_part = (double*)(ws + L.sumsq_part);
  Entry* coo_l = (Entry*)(ws + L.coo_l);

  uint64_t thresh = (uint64_t)std::floor(p * 4294967296.0);
  if (thresh > (1ull << 32)) thresh = 1ull << 32;

  hipLaunchKernelGGL(k_sample_init, dim3(1), dim3(64), 0, st, hdr, p, thresh, cap, seed, window,
                     (uint64_t)coin);
  if (coin)
    hipLaunchKernelGGL(k_sample_mask_ticks, dim3(si.nblk), dim3(kThreads), 0, st, si.N,
                       si.fdim[si.d - 1], thresh, (uint32_t)seed, (uint32_t)(seed >> 32), window,
                       bitmap, blkcnt);
  else
    hipLaunchKernelGGL(k_sample_mask, dim3(si.nblk), dim3(kThreads), 0, st, si.N, thresh,
                       (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)window,
                       (uint32_t)(window >> 32), bitmap, blkcnt);
  scan_u32(blkcnt, si.nblk, (uint32_t*)(ws + L.scan_tmp), st);
  if (x_is_f64)
    hipLaunchKernelGGL(k_sample_compact<double>, dim3(si.nblk), dim3(kThreads), 0, st,
                       (const double*)X, si.N, bitmap, blkcnt, wrank, coo_l, cap, sumsq_part);
  else
    hipLaunchKernelGGL(k_sample_compact<float>, dim3(si.nblk), dim3(kThreads), 0, st,
                       (const float*)X, si.N, bitmap, blkcnt, wrank, coo_l, cap, sumsq_part);
  return launch_layouts(si, ws, L, st);
}

hipError_t launch_sample_slide(const ShapeInfo& si, int x_is_f64, const void* X, double p,
                               uint64_t seed, uint64_t tick0, char* ws, const SampleLayout& L,
                               uint64_t cap, const char* ws_prev, hipStream_t st) {
  SampleHdr* hdr = (SampleHdr*)(ws + L.hdr);
  uint64_t* bitmap = (uint64_t*)(ws + L.bitmap);
  uint32_t* wrank = (uint32_t*)(ws + L.wrank);
  uint32_t* blkcnt = (uint32_t*)(ws + L.blkcnt);
  double* sumsq_part = (double*)(ws + L.sumsq_part);
  Entry* coo_l = (Entry*)(ws + L.coo_l);
  uint64_t thresh = (uint64_t)std::floor(p * 4294967296.0);
  if (thresh > (1ull << 32)) thresh = 1ull << 32;
  PrevSample pv{(const SampleHdr*)(ws_prev + L.hdr), (const uint64_t*)(ws_prev + L.bitmap),
                (const uint32_t*)(ws_prev + L.wrank), (const Entry*)(ws_prev + L.coo_l)};
  hipLaunchKernelGGL(k_sample_init, dim3(1), dim3(64), 0, st, hdr, p, thresh, cap, seed, tick0,
                     (uint64_t)1);
  const FastDiv fT = si.fdim[si.d - 1];
  hipLaunchKernelGGL(k_sample_mask_slide, dim3(si.nblk), dim3(kThreads), 0, st, si.N, fT, thresh, seed,
                     tick0, cap, pv, bitmap, blkcnt);
  scan_u32(blkcnt, si.nblk, (uint32_t*)(ws + L.scan_tmp), st);
  hipLaunchKernelGGL(k_word_ranks, dim3(si.nblk), dim3(kThreads), 0, st, bitmap, blkcnt, wrank);
  const uint32_t T = si.dims[si.d - 1], nseries = si.N / T;
  if (!x_is_f64)
    hipLaunchKernelGGL(k_slide_copy_runs, dim3((nseries + 3) / 4), dim3(256), 0, st, nseries, T, tick0,
                       seed, thresh, cap, pv, bitmap, wrank, blkcnt + si.nblk, coo_l);
  if (x_is_f64)
    hipLaunchKernelGGL(k_sample_compact_slide<double>, dim3(si.nblk), dim3(kThreads), 0, st,
                       (const double*)X, si.N, fT, tick0, seed, thresh, pv, bitmap, blkcnt, wrank, coo_l,
                       cap, sumsq_part);
  else
    hipLaunchKernelGGL(k_sample_compact_slide<float>, dim3(si.nblk), dim3(kThreads), 0, st,
                       (const float*)X, si.N, fT, tick0, seed, thresh, pv, bitmap, blkcnt, wrank, coo_l,
                       cap, sumsq_part);
  return launch_layouts(si, ws, L, st);
}

// Kept count and status, then the CSR row pointers and the CSC copy.
hipError_t launch_layouts(const ShapeInfo& si, char* ws, const SampleLayout& L, hipStream_t st) {
  SampleHdr* hdr = (SampleHdr*)(ws + L.hdr);
  uint64_t* bitmap = (uint64_t*)(ws + L.bitmap);
  uint32_t* wrank = (uint32_t*)(ws + L.wrank);
  uint32_t* blkcnt = (uint32_t*)(ws + L.blkcnt);
  double* sumsq_part = (double*)(ws + L.sumsq_part);
  Entry* coo_l = (Entry*)(ws + L.coo_l);
  uint32_t* rowptr = (uint32_t*)(ws + L.rowptr);
  uint32_t* colptr = (uint32_t*)(ws + L.colptr);
  uint32_t* csc_cnt = (uint32_t*)(ws + L.csc_cnt);
  uint32_t* headrow = (uint32_t*)(ws + L.headrow);
  Entry* coo_t = (Entry*)(ws + L.coo_t);
  hipLaunchKernelGGL(k_sample_finalize, dim3(1), dim3(256), 0, st, hdr, blkcnt, si.nblk,
                     sumsq_part, wrank, si.nwords);
  hipLaunchKernelGGL(k_rowptr, dim3((si.MH + 1 + 255) / 256), dim3(256), 0, st, si, bitmap,
                     wrank, hdr, rowptr);
  hipLaunchKernelGGL(k_headrow, dim3((si.MH + 255) / 256), dim3(256), 0, st, si, headrow,
                     (uint32_t*)(ws + L.headpos));
  dim3 g((si.MT + 63) / 64, (si.nrb + 3) / 4);
  hipLaunchKernelGGL(k_csc_count, g, dim3(256), 0, st, si, bitmap, headrow, csc_cnt);
  scan_u32(csc_cnt, si.MT * si.nrb, (uint32_t*)(ws + L.scan_tmp), st);
  hipLaunchKernelGGL(k_csc_fill, g, dim3(256), 0, st, si, bitmap, wrank, headrow, csc_cnt, coo_l,
                     coo_t, colptr, (uint32_t*)(ws + L.cscpos), hdr);
  return hipGetLastError();
}

}  // namespace mach
