// Sparse tensor-times-matrix chain (Alg. 2, the "Y <-" line; the n-mode
// product of Section 2.1) without float atomics.
//
// A segment is one CSR row (head index r, entries ordered by tail
// coordinates) or one CSC column (tail index c, entries ordered by head
// coordinates).  For each segment the kernel forms
//     out[seg, kappa] = sum_{entries z} v_z * prod_{contracted k} A_k[i_k(z), j_k]
// with at most two contracted modes, evaluated fiber by fiber: along the
// inner contracted mode it accumulates t = sum v * A_in[i_in, :] (R_in
// values); when the outer coordinate changes it adds A_out[i_out, :] (x) t
// into s (R_out x R_in values).  Each segment is split into G contiguous
// sub-ranges, one per lane, so every lane walks whole fibers in registers;
// the G partial results are then summed by a fixed xor butterfly.  The
// result depends only on the data, never on scheduling.
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
  const float* Ain;        // inner factor, row stride 16, zero padded
  const float* Aout;       // outer factor (two contracted modes only)
  uint32_t Rin, Rout;
  float* out;              // out[seg * K + kappa]
  uint32_t K;
  int G;                   // lanes per segment (power of two, 4..64)
  const SampleHdr* hdr;
  const int32_t* st_solver;
};

template <int NQ, int RI, int RO>
__global__ __launch_bounds__(256) void k_spc(SpcArgs a) {
  if (a.hdr->status != 0 || *a.st_solver != 0) return;
  const int G = a.G;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const uint32_t seg = blockIdx.x * (256u / G) + threadIdx.x / G;
  const bool valid = seg < a.nseg;
  uint32_t lo = 0, hi = 0;
  if (valid) {
    uint32_t b0 = a.segptr[seg], b1 = a.segptr[seg + 1];
    uint32_t L = b1 - b0;
    lo = b0 + (uint32_t)(((uint64_t)L * gl) / G);
    hi = b0 + (uint32_t)(((uint64_t)L * (gl + 1)) / G);
  }
  constexpr int NS = (NQ == 2) ? RO * RI : RI;
  float t[RI];
  float s[NS];
#pragma unroll
  for (int j = 0; j < RI; ++j) t[j] = 0.f;
#pragma unroll
  for (int j = 0; j < NS; ++j) s[j] = 0.f;
  uint32_t cur = 0xffffffffu;
  const uint32_t segbase = seg * a.MT;
  // Batches of U entries: all loads of a batch are issued before any use,
  // so each lane waits for memory once per batch rather than per entry.
  constexpr int U = (NS + 4 * RI <= 160) ? 4 : 2;
  for (uint32_t e0 = lo; e0 < hi; e0 += U) {
    Entry en[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u < hi) {
        en[u] = a.ent[e0 + u];
      } else {
        en[u].l = a.csc ? 0u : segbase;
        en[u].v = 0.f;
      }
    }
    uint32_t iin[U], iout[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t x = a.csc ? a.fMT.div(en[u].l) : en[u].l - segbase;
      iin[u] = x;
      iout[u] = 0;
      if (NQ == 2) {
        uint32_t h = a.flo.div(x);
        uint32_t l = x - h * a.flo.d;
        iin[u] = a.inner_is_lo ? l : h;
        iout[u] = a.inner_is_lo ? h : l;
      }
    }
    float4 w[U][RI / 4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float4* ap = reinterpret_cast<const float4*>(a.Ain + (size_t)iin[u] * 16);
#pragma unroll
      for (int q = 0; q < RI / 4; ++q) w[u][q] = ap[q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (NQ == 2 && e0 + u < hi && iout[u] != cur) {
        if (cur != 0xffffffffu) {
          const float* ao = a.Aout + (size_t)cur * 16;
#pragma unroll
          for (int o = 0; o < RO; ++o) {
            float wo = ao[o];
#pragma unroll
            for (int j = 0; j < RI; ++j) s[o * RI + j] = fmaf(wo, t[j], s[o * RI + j]);
          }
#pragma unroll
          for (int j = 0; j < RI; ++j) t[j] = 0.f;
        }
        cur = iout[u];
      }
      const float v = en[u].v;
#pragma unroll
      for (int q = 0; q < RI / 4; ++q) {
        t[4 * q + 0] = fmaf(v, w[u][q].x, t[4 * q + 0]);
        t[4 * q + 1] = fmaf(v, w[u][q].y, t[4 * q + 1]);
        t[4 * q + 2] = fmaf(v, w[u][q].z, t[4 * q + 2]);
        t[4 * q + 3] = fmaf(v, w[u][q].w, t[4 * q + 3]);
      }
    }
  }
  if (NQ == 2) {
    if (cur != 0xffffffffu) {
      const float* ao = a.Aout + (size_t)cur * 16;
#pragma unroll
      for (int o = 0; o < RO; ++o) {
        float w = ao[o];
#pragma unroll
        for (int j = 0; j < RI; ++j) s[o * RI + j] = fmaf(w, t[j], s[o * RI + j]);
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < RI; ++j) s[j] = t[j];
  }
  // Sum the G lanes of the segment (fixed butterfly order).
  for (int m = 1; m < G; m <<= 1) {
#pragma unroll
    for (int j = 0; j < NS; ++j) s[j] += __shfl_xor(s[j], m, 64);
  }
  if (!valid) return;
  float* o = a.out + (size_t)seg * a.K;
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    if ((u & (G - 1)) != gl) continue;
    uint32_t jo = (NQ == 2) ? (uint32_t)(u / RI) : 0u, ji = (uint32_t)(u % RI);
    if (ji >= a.Rin || jo >= (NQ == 2 ? a.Rout : 1u)) continue;
    uint32_t kappa = (NQ == 2) ? (a.inner_is_lo ? jo * a.Rin + ji : ji * a.Rout + jo) : ji;
    o[kappa] = s[u];
  }
}

inline int pad4(uint32_t r) { return r <= 4 ? 4 : r <= 8 ? 8 : r <= 12 ? 12 : 16; }

template <int NQ, int RI, int RO>
hipError_t go(const SpcArgs& a, hipStream_t st) {
  uint32_t per = 256u / a.G;
  dim3 grid((a.nseg + per - 1) / per);
  hipEvent_t e0, e1;
  if (timing_events(a.csc, &e0, &e1))
    hipExtLaunchKernelGGL((k_spc<NQ, RI, RO>), grid, dim3(256), 0, st, e0, e1, 0, a);
  else
    hipLaunchKernelGGL((k_spc<NQ, RI, RO>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int NQ, int RI>
hipError_t go_ro(const SpcArgs& a, hipStream_t st) {
  if constexpr (NQ == 1) {
    return go<NQ, RI, 1>(a, st);
  } else {
    switch (pad4(a.Rout)) {
      case 4: return go<NQ, RI, 4>(a, st);
      case 8: return go<NQ, RI, 8>(a, st);
      case 12: return go<NQ, RI, 12>(a, st);
      default: return go<NQ, RI, 16>(a, st);
    }
  }
}

template <int NQ>
hipError_t go_ri(const SpcArgs& a, hipStream_t st) {
  switch (pad4(a.Rin)) {
    case 4: return go_ro<NQ, 4>(a, st);
    case 8: return go_ro<NQ, 8>(a, st);
    case 12: return go_ro<NQ, 12>(a, st);
    default: return go_ro<NQ, 16>(a, st);
  }
}

int lanes_per_segment(double density, uint32_t dense_len) {
  double est = density * (double)dense_len;
  int G = 4;
  while (G < 64 && (double)(2 * G) * 8.0 <= est) G *= 2;
  return G;
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

hipError_t launch_contract_tail(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                char* ws, const int32_t* ranks, double density, hipStream_t st) {
  SpcArgs a{};
  a.ent = sp.coo_l;
  a.segptr = sp.rowptr;
  a.nseg = si.MH;
  a.csc = 0;
  a.MT = si.MT;
  a.fMT = si.fMT;
  int q = si.d - si.h;
  a.Ain = (const float*)(ws + SL.af[si.d - 1]);
  a.Rin = ranks[si.d - 1];
  if (q == 2) {
    a.flo = si.fdim[si.d - 1];
    a.inner_is_lo = 1;
    a.Aout = (const float*)(ws + SL.af[si.h]);
    a.Rout = ranks[si.h];
  } else {
    a.flo = make_fastdiv(1);
    a.Aout = a.Ain;
    a.Rout = 1;
  }
  a.out = (float*)(ws + SL.TH);
  a.K = SL.KT;
  a.G = lanes_per_segment(density, si.MT);
  a.hdr = sp.hdr;
  a.st_solver = (const int32_t*)(ws + SL.status);
  return q == 2 ? go_ri<2>(a, st) : go_ri<1>(a, st);
}

hipError_t launch_contract_head(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                char* ws, const int32_t* ranks, double density, hipStream_t st) {
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
    a.Ain = (const float*)(ws + SL.af[inner]);
    a.Rin = ranks[inner];
    a.Aout = (const float*)(ws + SL.af[outer]);
    a.Rout = ranks[outer];
  } else {
    a.flo = make_fastdiv(1);
    a.Ain = (const float*)(ws + SL.af[0]);
    a.Rin = ranks[0];
    a.Aout = a.Ain;
    a.Rout = 1;
  }
  a.out = (float*)(ws + SL.TT);
  a.K = SL.KH;
  a.G = lanes_per_segment(density, si.MH);
  a.hdr = sp.hdr;
  a.st_solver = (const int32_t*)(ws + SL.status);
  return q == 2 ? go_ri<2>(a, st) : go_ri<1>(a, st);
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
