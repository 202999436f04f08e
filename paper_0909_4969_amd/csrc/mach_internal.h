// Internal definitions shared by the HIP kernels and the C-ABI layer.
// Nothing here is part of the public interface (include/mach.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mach.h"

#define MACH_HD __host__ __device__ __forceinline__

namespace mach {

// ---------------------------------------------------------------------------
// Division of uint32 by a run-time invariant divisor: one mulhi, one sub, two
// shifts (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI'94; the round-up variant with a 33-bit multiplier
// folded into an add-and-halve step).
// ---------------------------------------------------------------------------
struct FastDiv {
  uint32_t d, m, s1, s2;
  MACH_HD uint32_t div(uint32_t n) const {
    uint32_t t = (uint32_t)(((uint64_t)n * m) >> 32);
    return (t + ((n - t) >> s1)) >> s2;
  }
  MACH_HD uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < (uint64_t)d) ++l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - (uint64_t)d)) / (uint64_t)d + 1ull);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 0 ? l - 1 : 0;
  return f;
}

// ---------------------------------------------------------------------------
// Shape description.  The tensor is split into "head" modes 0..h-1 and
// "tail" modes h..d-1.  With r = head row index (C order over head modes)
// and c = tail column index (C order over tail modes), the linear index is
// l = r * MT + c: the kept entries in l order form a CSR matrix of MH rows
// and MT columns.  A second copy, sorted by (c, head coordinates in the
// order headperm), is its CSC form.
// ---------------------------------------------------------------------------
constexpr int kMaxD = MACH_MAX_D;
constexpr int kMaxRank = 16;      // largest R_n the sweep kernels handle
constexpr int kSmallEig = 64;     // largest side of the one-workgroup Jacobi

struct ShapeInfo {
  int32_t d, h;
  uint32_t N, MH, MT;
  uint32_t dims[kMaxD];
  uint32_t stride[kMaxD];         // C-order strides of the full tensor
  FastDiv fdim[kMaxD];
  FastDiv fstride[kMaxD];
  FastDiv fMT;
  int32_t headperm[kMaxD];        // CSC head order, outermost first (length h)
  uint32_t nblk;                  // sampler blocks of kSampleBlockElems
  uint32_t nwords;                // bitmap words = nblk * 256
  uint32_t nrb;                   // CSC row blocks
  uint32_t rb;                    // rows per CSC row block
};

constexpr uint32_t kSampleBlockElems = 16384;   // 256 words of 64 bits
constexpr uint32_t kSampleBlockWords = 256;

// Device-resident header at offset 0 of the sample workspace.
struct SampleHdr {
  uint64_t nnz;          // kept entries (may exceed cap)
  uint64_t cap;
  double p;
  double sumsq;          // sum of kept x^2 (unscaled)
  uint64_t thresh;       // keep iff word < thresh
  uint64_t seed, window;  // window: the window id, or the first tick (tick-keyed coins)
  int32_t status;
  int32_t magic;
  uint64_t coin;         // 0: coins keyed by (seed, window) on l; 1: by (seed, series, tick)
  uint64_t pad[6];
};
constexpr int32_t kSampleMagic = 0x4d414348;   // "MACH"

struct SampleLayout {
  size_t hdr, bitmap, wrank, blkcnt, sumsq_part, coo_l, rowptr, colptr,
      csc_cnt, headrow, coo_t, scan_tmp, cscpos, headpos, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Returns false if the shape is invalid or unsupported.
bool make_shape_info(const mach_shape* s, ShapeInfo* out);
SampleLayout sample_layout(const ShapeInfo& si, uint64_t cap);

// Kept entry: linear index and the float32 input value (not divided by p).
struct __align__(8) Entry {
  uint32_t l;
  float v;
};

// Rank of bit l in the bitmap: number of kept entries with index < l.
__device__ __forceinline__ uint32_t bit_rank(const uint64_t* bitmap, const uint32_t* wrank,
                                             uint32_t l) {
  uint32_t w = l >> 6, b = l & 63;
  uint64_t word = bitmap[w];
  uint64_t lo = b ? (word & ((~0ull) >> (64 - b))) : 0ull;
  return wrank[w] + (uint32_t)__popcll(lo);
}

// ---------------------------------------------------------------------------
// Kernel launchers (one per .hip file).  All return hipError_t of the launch.
// ---------------------------------------------------------------------------
hipError_t launch_sample(const ShapeInfo& si, int x_is_f64, const void* X, double p,
                         uint64_t seed, uint64_t window, char* ws, const SampleLayout& L,
                         uint64_t cap, hipStream_t st, int coin = 0);
// Tick-keyed toss of a window from an earlier window's sample (same layout).
hipError_t launch_sample_slide(const ShapeInfo& si, int x_is_f64, const void* X, double p,
                               uint64_t seed, uint64_t tick0, char* ws, const SampleLayout& L,
                               uint64_t cap, const char* ws_prev, hipStream_t st);
// Kept count, status and the CSR / CSC layouts of a tossed sample.
hipError_t launch_layouts(const ShapeInfo& si, char* ws, const SampleLayout& L, hipStream_t st);

}  // namespace mach
