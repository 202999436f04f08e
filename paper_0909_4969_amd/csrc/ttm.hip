// Sparse tensor-times-matrix chain (the projection of the tensor onto all
// factors but one in Alg. 2; the n-mode product of Section 2.1) without
// float atomics.
//
// A segment is one CSR row (head index r, entries ordered by tail
// coordinates) or one CSC column (tail index c, entries ordered by head
// coordinates).  For each segment the kernel forms
//     out[seg, kappa] = sum_{entries z} v_z * prod_{contracted k} A_k[i_k(z), j_k]
// with at most two contracted modes, evaluated fiber by fiber: along the
// inner contracted mode it accumulates t = sum v * A_in[i_in, :] (R_in
// values); when the outer coordinate changes it adds A_out[i_out, :] (x) t
// into s (R_out x R_in values).  The entries of a segment are dealt to S
// slots (contiguous sub-ranges when fibers must stay whole, else strided);
// a slot is R_in / 4 lanes that each own four inner columns.  The S partial
// results are summed by a fixed xor butterfly, so the result depends only
// on the data, never on scheduling.
#include <hip/hip_ext.h>

#include "solver.h"

namespace mach {
namespace {

struct SpcArgs {
  const Entry* ent;
  const uint32_t* segptr;
  uint32_t nseg;
  int csc;                 // 1: x = l / MT (head row); 0: x = l - seg * MT (tail column)
  uint32_t MT;
  FastDiv fMT, flo;        // flo divides x into (hi, lo) contracted coordinates
  int inner_is_lo;
  const void* Ain;         // inner factor, row stride 16, zero padded (float32 or bfloat16)
  const void* Aout;        // outer factor (two contracted modes only)
  uint32_t Rin, Rout;
  uint32_t nin, nout;      // rows of Ain and Aout
  float* out;              // out[seg * K + kappa]
  uint32_t K;
  int G;                   // lanes per segment (power of two, 1..256)
  double density;          // expected kept fraction, and the dense length of a segment
  uint32_t dense_len;
  const SampleHdr* hdr;
  const int32_t* st_solver;
};

// Entries of the workgroup's segments are staged through LDS in chunks of
// kStage: one coalesced non-temporal pass over the entry stream (it is read
// once per sweep, so it should not evict the factor rows from L2).
constexpr uint32_t kStage = 4096;

// Lane layout: LPE = RI / 4 lanes share one entry, lane `quad` owning inner
// columns 4*quad .. 4*quad+3, so the LPE lanes gather one contiguous 16*LPE
// byte factor row together (one cache line per entry instead of one per
// lane and float4).  The G lanes of a segment form S = G / LPE entry slots.
// Four factor entries (columns 4 quad .. 4 quad + 3 of a row) as float32,
// from float32 or bfloat16 (BF) storage.
template <int BF>
__device__ __forceinline__ float4 factor4(const void* A, size_t row, int quad) {
  if constexpr (BF) {
    const uint2 u = reinterpret_cast<const uint2*>(A)[row * 4 + quad];
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  } else {
    return reinterpret_cast<const float4*>(A)[row * 4 + quad];
  }
}

// LF = 1: the factors are small enough to be copied into LDS (as float32,
// the RI / 4 and RO / 4 used quads of each row) when the kernel starts, and
// every factor row is then read from there instead of gathered through L2.
constexpr uint32_t kLdsFactorBytes = 16384;

template <int NQ, int RI, int RO>
__host__ __device__ constexpr uint32_t lds_factor_bytes(uint32_t nin, uint32_t nout) {
  return (nin * (RI / 4) + (NQ == 2 ? nout * (RO / 4) : 0u)) * 16u;
}

template <int NQ, int RI, int RO, int CSC, int BF, int LF>
__global__ __launch_bounds__(256) void k_spc(SpcArgs a) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  constexpr int LPE = RI / 4;
  static_assert(LPE == 1 || LPE == 2 || LPE == 4, "RI must be 4, 8 or 16");
  __shared__ uint64_t stage[kStage];
  extern __shared__ float4 fsh[];   // LF: Ain rows (LPE quads each), then Aout rows (RO / 4 quads)
  if constexpr (LF) {
    const uint32_t nq_in = a.nin * LPE;
    for (uint32_t e = threadIdx.x; e < nq_in; e += 256) fsh[e] = factor4<BF>(a.Ain, e / LPE, e % LPE);
    if constexpr (NQ == 2)
      for (uint32_t e = threadIdx.x; e < a.nout * (RO / 4); e += 256)
        fsh[nq_in + e] = factor4<BF>(a.Aout, e / (RO / 4), e % (RO / 4));
    __syncthreads();
  }
  const float4* fin = fsh;
  const float4* fout = fsh + a.nin * LPE;
  const int G = a.G;
  const int S = G / LPE;
  const int gl = threadIdx.x & (G - 1);
  const int quad = gl & (LPE - 1);
  const int slot = gl / LPE;
  const uint32_t per = 256u / G;
  const uint32_t seg0 = blockIdx.x * per;
  const uint32_t seg = seg0 + threadIdx.x / G;
  const bool valid = seg < a.nseg;
  const uint32_t segN = min(a.nseg, seg0 + per);
  const uint32_t wg_lo = a.segptr[seg0], wg_hi = a.segptr[segN];
  uint32_t b0 = 0, b1 = 0;
  if (valid) {
    b0 = a.segptr[seg];
    b1 = a.segptr[seg + 1];
  }
  // Two contracted modes: slot walks the contiguous sub-range [lo, hi) (whole
  // fibers stay in one slot).  One contracted mode: slot takes entries
  // b0 + slot, b0 + slot + S, ... (order is irrelevant to a plain sum).
  uint32_t lo = b0, hi = b1;
  if (NQ == 2) {
    uint32_t L = b1 - b0;
    lo = b0 + (uint32_t)(((uint64_t)L * slot) / S);
    hi = b0 + (uint32_t)(((uint64_t)L * (slot + 1)) / S);
  }
  constexpr int NS = (NQ == 2) ? RO * 4 : 4;
  float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
  float s[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) s[j] = 0.f;
  uint32_t cur = 0xffffffffu;
  const uint32_t segbase = seg * a.MT;
  // The next chunk is fetched into registers (all kPer loads issued back to
  // back) while the current one is processed.
  constexpr int kPer = kStage / 256;
  const uint64_t* ent64 = reinterpret_cast<const uint64_t*>(a.ent);
  uint64_t nxt[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t e = wg_lo + threadIdx.x + k * 256;
    nxt[k] = e < wg_hi ? __builtin_nontemporal_load(ent64 + e) : 0ull;
  }
  for (uint32_t c0 = wg_lo; c0 < wg_hi; c0 += kStage) {
    const uint32_t c1 = min(wg_hi, c0 + kStage);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) stage[threadIdx.x + k * 256] = nxt[k];
    __syncthreads();
    if (c1 < wg_hi) {
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const uint32_t e = c1 + threadIdx.x + k * 256;
        nxt[k] = e < wg_hi ? __builtin_nontemporal_load(ent64 + e) : 0ull;
      }
    }
    uint32_t e_begin, e_step;
    if (NQ == 2) {
      e_begin = max(lo, c0);
      e_step = 1;
    } else {
      uint32_t first = b0 + slot;
      e_begin = first >= c0 ? first : first + ((c0 - first + S - 1) / S) * S;
      e_step = S;
    }
    const uint32_t e_end = NQ == 2 ? min(hi, c1) : min(b1, c1);
    // U entries per step, straight-line code: all U factor rows are requested
    // before any is used (an entry past the end re-reads entry e, weight 0).
    constexpr int U = NQ == 2 ? 4 : 8;
    for (uint32_t e = e_begin; e < e_end; e += U * e_step) {
      float4 w[U];
      float v[U];
      uint32_t io[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t eu = e + u * e_step;
        const bool ok = eu < e_end;
        const uint64_t en = stage[(ok ? eu : e) - c0];
        const uint32_t el = (uint32_t)en;
        v[u] = ok ? __uint_as_float((uint32_t)(en >> 32)) : 0.f;
        const uint32_t x = CSC ? a.fMT.div(el) : el - segbase;
        uint32_t iin = x;
        io[u] = 0xffffffffu;
        if (NQ == 2) {
          uint32_t h = a.flo.div(x);
          uint32_t l = x - h * a.flo.d;
          iin = a.inner_is_lo ? l : h;
          io[u] = ok ? (a.inner_is_lo ? h : l) : 0xffffffffu;
        }
        w[u] = LF ? fin[iin * LPE + quad] : factor4<BF>(a.Ain, iin, quad);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (NQ == 2 && io[u] != 0xffffffffu && io[u] != cur) {
          if (cur != 0xffffffffu) {
#pragma unroll
            for (int o4 = 0; o4 < RO / 4; ++o4) {
              const float4 wo = LF ? fout[cur * (RO / 4) + o4] : factor4<BF>(a.Aout, cur, o4);
              const float wv[4] = {wo.x, wo.y, wo.z, wo.w};
#pragma unroll
              for (int oo = 0; oo < 4; ++oo) {
                float* so = s + (o4 * 4 + oo) * 4;
                so[0] = fmaf(wv[oo], t.x, so[0]);
                so[1] = fmaf(wv[oo], t.y, so[1]);
                so[2] = fmaf(wv[oo], t.z, so[2]);
                so[3] = fmaf(wv[oo], t.w, so[3]);
              }
            }
            t = make_float4(0.f, 0.f, 0.f, 0.f);
          }
          cur = io[u];
        }
        t.x = fmaf(v[u], w[u].x, t.x);
        t.y = fmaf(v[u], w[u].y, t.y);
        t.z = fmaf(v[u], w[u].z, t.z);
        t.w = fmaf(v[u], w[u].w, t.w);
      }
    }
  }
  if (NQ == 2) {
    if (cur != 0xffffffffu) {
#pragma unroll
      for (int o4 = 0; o4 < RO / 4; ++o4) {
        const float4 wo = LF ? fout[cur * (RO / 4) + o4] : factor4<BF>(a.Aout, cur, o4);
        const float wv[4] = {wo.x, wo.y, wo.z, wo.w};
#pragma unroll
        for (int oo = 0; oo < 4; ++oo) {
          float* so = s + (o4 * 4 + oo) * 4;
          so[0] = fmaf(wv[oo], t.x, so[0]);
          so[1] = fmaf(wv[oo], t.y, so[1]);
          so[2] = fmaf(wv[oo], t.z, so[2]);
          so[3] = fmaf(wv[oo], t.w, so[3]);
        }
      }
    }
  } else {
    s[0] = t.x;
    s[1] = t.y;
    s[2] = t.z;
    s[3] = t.w;
  }
  // Sum the S slots of the segment: a fixed xor butterfly within each wave,
  // then (segments wider than a wave) the wave sums in wave order via LDS.
  const int GW = G < 64 ? G : 64;
  for (int m = LPE; m < GW; m <<= 1) {
#pragma unroll
    for (int j = 0; j < NS; ++j) s[j] += __shfl_xor(s[j], m, 64);
  }
  if (G > 64) {
    __shared__ float red[4][4][NS];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < LPE)
#pragma unroll
      for (int j = 0; j < NS; ++j) red[wv][quad][j] = s[j];
    __syncthreads();
    if (gl < LPE)
      for (int w2 = 1; w2 < G / 64; ++w2)
#pragma unroll
        for (int j = 0; j < NS; ++j) s[j] += red[wv + w2][quad][j];
  }
  if (!valid || slot != 0) return;
  float* o = a.out + (size_t)seg * a.K;
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const uint32_t jo = (NQ == 2) ? (uint32_t)(u / 4) : 0u;
    const uint32_t ji = (uint32_t)(quad * 4 + (u & 3));
    if (ji >= a.Rin || jo >= (NQ == 2 ? a.Rout : 1u)) continue;
    const uint32_t kappa = (NQ == 2) ? (a.inner_is_lo ? jo * a.Rin + ji : ji * a.Rout + jo) : ji;
    o[kappa] = s[u];
  }
}

// ---------------------------------------------------------------------------
// Head-row pass with one contracted tail mode whose factor is too large for
// LDS (a long time mode): TH[r, :] = sum over the kept entries (r, c) of
// v * A[c, :].  The rows x columns plane is cut into tiles of RB head rows
// by TC tail columns.  A workgroup copies the TC factor rows of its tile into
// LDS once, so a factor row is fetched from L2 once per tile instead of once
// per kept entry.  Each row of the tile belongs to LPE lanes (lane `quad`
// owns inner columns 4 quad .. 4 quad + 3); its entries with c0 <= c < c1
// (found by two bitmap ranks) are loaded by those lanes together, kLoad per
// lane and all in flight at once, then passed round the LPE lanes by DPP
// quad permutes, and each entry's factor row is read from LDS.  Every tile
// writes one partial row per head row, and k_rows_tiled_sum adds the
// partials of a row in tile order: the result does not depend on
// scheduling, and no float atomics are used.
// ---------------------------------------------------------------------------
struct TiledArgs {
  const Entry* ent;            // kept entries in linear-index order
  const uint64_t* bitmap;
  const uint32_t* wrank;
  uint32_t MH, MT;
  const void* F;               // tail factor copy, row stride 16 (float32 or bfloat16)
  uint32_t Rin;                // used factor columns
  uint32_t TC, nT, RB;         // ticks per tile, tiles, rows per block
  float4* part;                // nT x MH x LPE float4 partial rows
  float* out;                  // TH, row stride K
  uint32_t K;
  const SampleHdr* hdr;
  const int32_t* st_solver;
};

// Kept entries with linear index below l (bit_rank, without reading the
// word past the bitmap when l is a multiple of 64).
__device__ __forceinline__ uint32_t rank_below(const uint64_t* bitmap, const uint32_t* wrank,
                                               uint32_t l) {
  return (l & 63u) ? bit_rank(bitmap, wrank, l) : wrank[l >> 6];
}

// Value of lane (lane & ~(LPE-1)) + src of the LPE-lane group (LPE = 1, 2, 4).
template <int LPE>
__device__ __forceinline__ uint32_t group_bcast(uint32_t x, int src) {
  if constexpr (LPE == 1) {
    return x;
  } else if constexpr (LPE == 2) {
    // quad_perm(src, src, 2 + src, 2 + src)
    return src == 0 ? (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xA0, 0xf, 0xf, false)
                    : (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xF5, 0xf, 0xf, false);
  } else {
    // quad_perm(src, src, src, src)
    switch (src) {
      case 0: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x00, 0xf, 0xf, false);
      case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x55, 0xf, 0xf, false);
      case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xAA, 0xf, 0xf, false);
      default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xFF, 0xf, 0xf, false);
    }
  }
}

constexpr int kLoad = 16;   // entry loads in flight per lane

template <int RI, int BF>
__global__ __launch_bounds__(256) void k_rows_tiled(TiledArgs a) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  constexpr int LPE = RI / 4;
  extern __shared__ float4 ftile[];          // TC rows x LPE quads
  const uint32_t tile = blockIdx.x, blk = blockIdx.y;
  const uint32_t c0 = tile * a.TC, c1 = min(a.MT, c0 + a.TC);
  const int quad = threadIdx.x & (LPE - 1);
  const uint32_t r_lo = blk * a.RB, r_hi = min(a.MH, r_lo + a.RB);
  // Ranks of the first rows are requested before the factor tile is copied.
  uint32_t r = r_lo + threadIdx.x / LPE;
  uint32_t lo = 0, hi = 0;
  if (r < r_hi) {
    lo = rank_below(a.bitmap, a.wrank, r * a.MT + c0);
    hi = rank_below(a.bitmap, a.wrank, r * a.MT + c1);
  }
  const uint32_t nq = (c1 - c0) * LPE;
  for (uint32_t e = threadIdx.x; e < nq; e += 256) ftile[e] = factor4<BF>(a.F, c0 + e / LPE, e % LPE);
  __syncthreads();
  const uint64_t* ent64 = reinterpret_cast<const uint64_t*>(a.ent);
  for (; r < r_hi; r += 256 / LPE) {
    if (r != r_lo + threadIdx.x / LPE) {
      lo = rank_below(a.bitmap, a.wrank, r * a.MT + c0);
      hi = rank_below(a.bitmap, a.wrank, r * a.MT + c1);
    }
    const uint32_t base = r * a.MT + c0;
    // an unused slot holds (base, 0.0f): column c0 with weight 0
    const uint64_t dummy = (uint64_t)base;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t e0 = lo; e0 < hi; e0 += LPE * kLoad) {
      uint64_t en[kLoad];
#pragma unroll
      for (int j = 0; j < kLoad; ++j) {
        const uint32_t e = e0 + LPE * j + quad;
        en[j] = e < hi ? ent64[e] : dummy;
      }
      // Step j holds entries e0 + LPE j .. e0 + LPE j + LPE - 1, of which
      // some exist only while LPE j < hi - e0.  The test is the same in the
      // LPE lanes of a row (a broadcast never reads a masked lane), and a
      // wave skips the step once every row in it is done, instead of
      // reading factor rows from LDS for weight-0 slots.
      const uint32_t left = hi - e0;
#pragma unroll
      for (int j = 0; j < kLoad; ++j) {
        if ((uint32_t)(LPE * j) >= left) continue;
#pragma unroll
        for (int q = 0; q < LPE; ++q) {
          const uint32_t l = group_bcast<LPE>((uint32_t)en[j], q);
          const float v = __uint_as_float(group_bcast<LPE>((uint32_t)(en[j] >> 32), q));
          const float4 w = ftile[(l - base) * LPE + quad];
          acc.x = fmaf(v, w.x, acc.x);
          acc.y = fmaf(v, w.y, acc.y);
          acc.z = fmaf(v, w.z, acc.z);
          acc.w = fmaf(v, w.w, acc.w);
        }
      }
    }
    a.part[((size_t)tile * a.MH + r) * LPE + quad] = acc;
  }
}

// TH[r, 4 q .. 4 q + 3] = sum over the tiles of the partials, one wave per
// head row: lane (t, q) adds tiles t, t + 64/LPE, ... in order, then a fixed
// xor butterfly adds the lanes of equal q.
template <int RI>
__global__ __launch_bounds__(256) void k_rows_tiled_sum(TiledArgs a) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  constexpr int LPE = RI / 4;
  constexpr uint32_t TS = 64 / LPE;       // tile lanes per row
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.MH) return;
  const uint32_t lane = threadIdx.x & 63, q = lane % LPE, t0 = lane / LPE;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  constexpr int U = 4;
  for (uint32_t t = t0; t < a.nT; t += U * TS) {
    float4 pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t tt = t + u * TS;
      pv[u] = tt < a.nT ? a.part[((size_t)tt * a.MH + r) * LPE + q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s.x += pv[u].x;
      s.y += pv[u].y;
      s.z += pv[u].z;
      s.w += pv[u].w;
    }
  }
  for (int m = LPE; m < 64; m <<= 1) {
    s.x += __shfl_xor(s.x, m, 64);
    s.y += __shfl_xor(s.y, m, 64);
    s.z += __shfl_xor(s.z, m, 64);
    s.w += __shfl_xor(s.w, m, 64);
  }
  if (t0 != 0) return;
  float* o = a.out + (size_t)r * a.K + 4 * q;
  const float sv[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (4 * q + j < a.Rin) o[j] = sv[j];
}

// Rows per block: 256 / LPE (one row per lane group) when a factor row
// copied into LDS then serves several kept entries (at least 3 expected);
// else 0 and the gather pass is used (sparse samples).
inline uint32_t tiled_rows_per_block(double density, int lpe) {
  const uint32_t rb = 256u / (uint32_t)lpe;
  return density * rb >= 3.0 ? rb : 0u;
}

template <int RI, int BF>
hipError_t go_tiled(TiledArgs a, hipStream_t st) {
  // Ticks per tile: the largest of 256 and 128 that still gives at least
  // 1024 workgroups (or the smallest).  Tiles of 256 (2048 workgroups on the
  // monitoring window) beat 512 and 1024 in spite of twice the partial rows.
  const uint32_t nrb = (a.MH + a.RB - 1) / a.RB;
  uint32_t tc = kTileTicksMax;
  while (tc > kTileTicksMin && (size_t)nrb * ((a.MT + tc - 1) / tc) < 1024) tc /= 2;
  a.TC = tc;
  a.nT = (a.MT + tc - 1) / tc;
  const uint32_t lds = tc * (RI / 4) * 16u;
  dim3 grid(a.nT, nrb);
  hipEvent_t e0, e1;
  const bool timed = timing_events(0, &e0, &e1);
  if (timed)
    hipExtLaunchKernelGGL((k_rows_tiled<RI, BF>), grid, dim3(256), lds, st, e0, nullptr, 0, a);
  else
    hipLaunchKernelGGL((k_rows_tiled<RI, BF>), grid, dim3(256), lds, st, a);
  const uint32_t nsum = (a.MH + 3) / 4;
  if (timed)
    hipExtLaunchKernelGGL((k_rows_tiled_sum<RI>), dim3(nsum), dim3(256), 0, st, nullptr, e1, 0, a);
  else
    hipLaunchKernelGGL((k_rows_tiled_sum<RI>), dim3(nsum), dim3(256), 0, st, a);
  return hipGetLastError();
}

inline int pad4(uint32_t r) { return r <= 4 ? 4 : r <= 8 ? 8 : r <= 12 ? 12 : 16; }

template <int NQ, int RI, int RO, int CSC, int BF, int LF>
hipError_t go_l(const SpcArgs& a, hipStream_t st) {
  uint32_t per = 256u / a.G;
  dim3 grid((a.nseg + per - 1) / per);
  const uint32_t lds = LF ? lds_factor_bytes<NQ, RI, RO>(a.nin, a.nout) : 0u;
  hipEvent_t e0, e1;
  if (timing_events(CSC, &e0, &e1))
    hipExtLaunchKernelGGL((k_spc<NQ, RI, RO, CSC, BF, LF>), grid, dim3(256), lds, st, e0, e1, 0, a);
  else
    hipLaunchKernelGGL((k_spc<NQ, RI, RO, CSC, BF, LF>), grid, dim3(256), lds, st, a);
  return hipGetLastError();
}

template <int NQ, int RI, int RO, int CSC, int BF>
hipError_t go_c(const SpcArgs& a, hipStream_t st) {
  if (lds_factor_bytes<NQ, RI, RO>(a.nin, a.nout) <= kLdsFactorBytes)
    return go_l<NQ, RI, RO, CSC, BF, 1>(a, st);
  return go_l<NQ, RI, RO, CSC, BF, 0>(a, st);
}

template <int NQ, int RI, int RO, int BF>
hipError_t go(const SpcArgs& a, hipStream_t st) {
  return a.csc ? go_c<NQ, RI, RO, 1, BF>(a, st) : go_c<NQ, RI, RO, 0, BF>(a, st);
}

template <int NQ, int RI, int BF>
hipError_t go_ro(const SpcArgs& a, hipStream_t st) {
  if constexpr (NQ == 1) {
    return go<NQ, RI, 1, BF>(a, st);
  } else {
    switch (pad4(a.Rout)) {
      case 4: return go<NQ, RI, 4, BF>(a, st);
      case 8: return go<NQ, RI, 8, BF>(a, st);
      case 12: return go<NQ, RI, 12, BF>(a, st);
      default: return go<NQ, RI, 16, BF>(a, st);
    }
  }
}

// Inner rank padded to 4, 8 or 16 (the lanes of one entry must be a power
// of two; factor rows are zero-padded to 16 columns, so 12 reads as 16).
inline int pad_inner(uint32_t r) { return r <= 4 ? 4 : r <= 8 ? 8 : 16; }

// Entry slots per segment: a power of two with an expected kSlotEntries
// entries or more per slot, such that the lanes per segment (slots times
// the lanes per entry, lpe) stay within kMaxSegLanes (a segment may span up
// to the four waves of a workgroup; one wave measured best on these passes).
constexpr double kSlotEntries = 16.0;
constexpr int kMaxSegLanes = 64;
int slots_per_segment(double density, uint32_t dense_len, int lpe) {
  double est = density * (double)dense_len;
  int S = 1;
  while (2 * S * lpe <= kMaxSegLanes && (double)(2 * S) * kSlotEntries <= est) S *= 2;
  return S;
}

template <int NQ, int BF>
hipError_t go_ri(SpcArgs a, hipStream_t st) {
  const int ri = pad_inner(a.Rin);
  a.G = slots_per_segment(a.density, a.dense_len, ri / 4) * (ri / 4);
  switch (ri) {
    case 4: return go_ro<NQ, 4, BF>(a, st);
    case 8: return go_ro<NQ, 8, BF>(a, st);
    default: return go_ro<NQ, 16, BF>(a, st);
  }
}

hipError_t go_any(const SpcArgs& a, int nq, int bf, hipStream_t st) {
  if (bf) return nq == 2 ? go_ri<2, 1>(a, st) : go_ri<1, 1>(a, st);
  return nq == 2 ? go_ri<2, 0>(a, st) : go_ri<1, 0>(a, st);
}

// bfloat16 copies (round to nearest even) of the float32 factor copies of
// the listed modes, for the mixed-precision sparse passes.
struct Bf16Args {
  const float* src[kMaxD];
  uint16_t* dst[kMaxD];
  uint32_t n[kMaxD];      // elements (I_k x 16)
  int count;
};

__global__ void k_factors_to_bf16(Bf16Args a, const SampleHdr* hdr) {
  if (hdr->status != 0) return;
  const int k = blockIdx.y;
  if (k >= a.count) return;
  const uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.n[k]) return;
  const uint32_t u = __float_as_uint(a.src[k][e]);
  a.dst[k][e] = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

hipError_t to_bf16(const ShapeInfo& si, const SolverLayout& SL, char* ws, int k0, int k1,
                   const SampleHdr* hdr, hipStream_t st) {
  Bf16Args b{};
  uint32_t nmax = 1;
  for (int k = k0; k < k1; ++k) {
    b.src[b.count] = (const float*)(ws + SL.af[k]);
    b.dst[b.count] = (uint16_t*)(ws + SL.af16[k]);
    b.n[b.count] = si.dims[k] * 16;
    if (b.n[b.count] > nmax) nmax = b.n[b.count];
    ++b.count;
  }
  hipLaunchKernelGGL(k_factors_to_bf16, dim3((nmax + 255) / 256, b.count), dim3(256), 0, st, b, hdr);
  return hipGetLastError();
}


// out[(o*R + r)*Q + q] = sum_i A[i*16 + r] * in[(o*I + i)*Q + q].  A
// workgroup owns 64 consecutive outputs; its 4 waves take every 4th i with
// two accumulators each, and the partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_dense_ttm(const float* __restrict__ in, uint32_t O, uint32_t I,
                                                   uint32_t Q, const float* __restrict__ A, uint32_t R,
                                                   float* __restrict__ out, const SampleHdr* hdr,
                                                   const int32_t* st_solver) {
  if (hdr->status != 0 || *st_solver != 0) return;
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t idx = (uint64_t)blockIdx.x * 64 + lane;
  const uint64_t total = (uint64_t)O * R * Q;
  float acc0 = 0.f, acc1 = 0.f;
  if (idx < total) {
    uint32_t q = (uint32_t)(idx % Q);
    uint64_t t = idx / Q;
    uint32_t r = (uint32_t)(t % R);
    uint32_t o = (uint32_t)(t / R);
    const float* src = in + (size_t)o * I * Q + q;
    uint32_t i = w;
    // four steps of the loop below at a time, their loads issued first (the
    // same additions in the same order)
    for (; i + 28 < I; i += 32) {
      float a[8], x[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[2 * u] = A[(size_t)(i + 8 * u) * 16 + r];
        x[2 * u] = src[(size_t)(i + 8 * u) * Q];
        a[2 * u + 1] = A[(size_t)(i + 8 * u + 4) * 16 + r];
        x[2 * u + 1] = src[(size_t)(i + 8 * u + 4) * Q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc0 = fmaf(a[2 * u], x[2 * u], acc0);
        acc1 = fmaf(a[2 * u + 1], x[2 * u + 1], acc1);
      }
    }
    for (; i + 4 < I; i += 8) {
      acc0 = fmaf(A[(size_t)i * 16 + r], src[(size_t)i * Q], acc0);
      acc1 = fmaf(A[(size_t)(i + 4) * 16 + r], src[(size_t)(i + 4) * Q], acc1);
    }
    if (i < I) acc0 = fmaf(A[(size_t)i * 16 + r], src[(size_t)i * Q], acc0);
  }
  red[w][lane] = acc0 + acc1;
  __syncthreads();
  if (w == 0 && idx < total) out[idx] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

struct F32Args {
  const double* A[kMaxD];
  float* af[kMaxD];
  uint32_t I[kMaxD], R[kMaxD];
  int d;
};

__global__ void k_factors_to_f32(F32Args a, const SampleHdr* hdr) {
  if (hdr->status != 0) return;
  int k = blockIdx.y;
  if (k >= a.d) return;
  uint32_t idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.I[k] * 16) return;
  uint32_t i = idx >> 4, j = idx & 15;
  a.af[k][idx] = j < a.R[k] ? (float)a.A[k][(size_t)i * a.R[k] + j] : 0.f;
}

}  // namespace

// TH = Xhat (unscaled, float32, C order) when the single tail mode is left
// uncompressed (its factor is the identity, so the head-row pass contracts
// nothing): one thread per bitmap word writes its 64 entries, the kept
// values taken in order from the word's rank.
__global__ __launch_bounds__(256) void k_densify(const uint64_t* __restrict__ bitmap,
                                                 const uint32_t* __restrict__ wrank,
                                                 const Entry* __restrict__ coo, uint32_t N,
                                                 float* __restrict__ out, const SampleHdr* hdr,
                                                 const int32_t* st_solver) {
  if (hdr->status != 0 || *st_solver != 0) return;
  const uint32_t w = blockIdx.x * 256 + threadIdx.x;
  const uint32_t l0 = w * 64u;
  if (l0 >= N) return;
  const uint64_t word = bitmap[w];
  uint32_t r = wrank[w];
#pragma unroll 4
  for (uint32_t b = 0; b < 64; b += 4) {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool kept = (word >> (b + k)) & 1ull;
      v[k] = kept ? coo[r].v : 0.f;
      r += kept ? 1u : 0u;
    }
    if (l0 + b + 3 < N) {
      *reinterpret_cast<float4*>(out + l0 + b) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (l0 + b + k < N) out[l0 + b + k] = v[k];
    }
  }
}

hipError_t launch_contract_tail(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                char* ws, const int32_t* ranks, double density, int bf16,
                                hipStream_t st) {
  if (SL.ident_last) {
    const uint32_t nw = (si.N + 63) / 64;
    hipLaunchKernelGGL(k_densify, dim3((nw + 255) / 256), dim3(256), 0, st, sp.bitmap, sp.wrank, sp.coo_l,
                       si.N, (float*)(ws + SL.TH), sp.hdr, (const int32_t*)(ws + SL.status));
    return hipGetLastError();
  }
  if (bf16) {
    hipError_t e = to_bf16(si, SL, ws, si.h, si.d, sp.hdr, st);
    if (e != hipSuccess) return e;
  }
  const size_t* fac = bf16 ? SL.af16 : SL.af;
  SpcArgs a{};
  a.ent = sp.coo_l;
  a.segptr = sp.rowptr;
  a.nseg = si.MH;
  a.csc = 0;
  a.MT = si.MT;
  a.fMT = si.fMT;
  int q = si.d - si.h;
  a.Ain = (const void*)(ws + fac[si.d - 1]);
  a.Rin = ranks[si.d - 1];
  a.nin = si.dims[si.d - 1];
  if (q == 2) {
    a.flo = si.fdim[si.d - 1];
    a.inner_is_lo = 1;
    a.Aout = (const void*)(ws + fac[si.h]);
    a.Rout = ranks[si.h];
    a.nout = si.dims[si.h];
  } else {
    a.flo = make_fastdiv(1);
    a.Aout = a.Ain;
    a.Rout = 1;
    a.nout = 0;
  }
  a.out = (float*)(ws + SL.TH);
  a.K = SL.KT;
  a.density = density;
  a.dense_len = si.MT;
  a.hdr = sp.hdr;
  a.st_solver = (const int32_t*)(ws + SL.status);
  const uint32_t rb = tiled_rows_per_block(density, pad_inner(a.Rin) / 4);
  if (q == 1 && SL.tpart && rb && (si.MH + rb - 1) / rb <= 65535u) {
    TiledArgs t{};
    t.ent = sp.coo_l;
    t.bitmap = sp.bitmap;
    t.wrank = sp.wrank;
    t.MH = si.MH;
    t.MT = si.MT;
    t.F = a.Ain;
    t.Rin = a.Rin;
    t.RB = rb;
    t.part = (float4*)(ws + SL.tpart);
    t.out = a.out;
    t.K = a.K;
    t.hdr = a.hdr;
    t.st_solver = a.st_solver;
    const int ri = pad_inner(a.Rin);
    if (bf16) return ri == 4 ? go_tiled<4, 1>(t, st) : ri == 8 ? go_tiled<8, 1>(t, st) : go_tiled<16, 1>(t, st);
    return ri == 4 ? go_tiled<4, 0>(t, st) : ri == 8 ? go_tiled<8, 0>(t, st) : go_tiled<16, 0>(t, st);
  }
  return go_any(a, q, bf16, st);
}

hipError_t launch_contract_head(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                char* ws, const int32_t* ranks, double density, int bf16,
                                hipStream_t st) {
  if (bf16) {
    hipError_t e = to_bf16(si, SL, ws, 0, si.h, sp.hdr, st);
    if (e != hipSuccess) return e;
  }
  const size_t* fac = bf16 ? SL.af16 : SL.af;
  SpcArgs a{};
  a.ent = sp.coo_t;
  a.segptr = sp.colptr;
  a.nseg = si.MT;
  a.csc = 1;
  a.MT = si.MT;
  a.fMT = si.fMT;
  int q = si.h;
  if (q == 2) {
    int inner = si.headperm[1], outer = si.headperm[0];
    a.flo = si.fdim[1];
    a.inner_is_lo = inner == 1;
    a.Ain = (const void*)(ws + fac[inner]);
    a.Rin = ranks[inner];
    a.nin = si.dims[inner];
    a.Aout = (const void*)(ws + fac[outer]);
    a.Rout = ranks[outer];
    a.nout = si.dims[outer];
  } else {
    a.flo = make_fastdiv(1);
    a.Ain = (const void*)(ws + fac[0]);
    a.Rin = ranks[0];
    a.nin = si.dims[0];
    a.Aout = a.Ain;
    a.Rout = 1;
    a.nout = 0;
  }
  a.out = (float*)(ws + SL.TT);
  a.K = SL.KH;
  a.density = density;
  a.dense_len = si.MH;
  a.hdr = sp.hdr;
  a.st_solver = (const int32_t*)(ws + SL.status);
  return go_any(a, q, bf16, st);
}

hipError_t launch_form_y(const ShapeInfo& si, const SolverLayout& SL, char* ws, int k,
                         const SampleHdr* hdr, hipStream_t st) {
  const ModePlan& m = SL.mp[k];
  if (m.contract_mode < 0) return hipSuccess;
  const float* src = (const float*)(ws + (k < si.h ? SL.TH : SL.TT));
  uint32_t R = SL.mp[m.contract_mode].R;
  uint64_t total = (uint64_t)m.cO * R * m.cQ;
  hipLaunchKernelGGL(k_dense_ttm, dim3((uint32_t)((total + 63) / 64)), dim3(256), 0, st, src, m.cO,
                     m.cI, m.cQ, (const float*)(ws + SL.af[m.contract_mode]), R,
                     (float*)(ws + m.ybuf), hdr, (const int32_t*)(ws + SL.status));
  return hipGetLastError();
}

hipError_t launch_factors_to_f32(const ShapeInfo& si, const SolverLayout& SL, char* ws,
                                 double* const* A, const int32_t* ranks, const SampleHdr* hdr,
                                 hipStream_t st) {
  F32Args a{};
  a.d = si.d;
  uint32_t imax = 0;
  for (int k = 0; k < si.d; ++k) {
    a.A[k] = A[k];
    a.af[k] = (float*)(ws + SL.af[k]);
    a.I[k] = si.dims[k];
    a.R[k] = ranks[k];
    if (si.dims[k] > imax) imax = si.dims[k];
  }
  hipLaunchKernelGGL(k_factors_to_f32, dim3((imax * 16 + 255) / 256, si.d), dim3(256), 0, st, a, hdr);
  return hipGetLastError();
}

}  // namespace mach
