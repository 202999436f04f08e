// C-ABI entry points (include/mach.h): argument validation, workspace
// layouts and launch sequencing.  Every device step runs in the kernels of
// the other .hip files; this file only checks, lays out and launches.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "mach_internal.h"
#include "solver.h"

namespace mach {

bool make_shape_info(const mach_shape* s, ShapeInfo* out) {
  if (!s || s->d < 2 || s->d > kMaxD) return false;
  ShapeInfo si;
  std::memset(&si, 0, sizeof(si));
  si.d = s->d;
  uint64_t N = 1;
  for (int k = 0; k < si.d; ++k) {
    if (s->dims[k] < 1 || s->dims[k] > (int64_t)0x7fffffff) return false;
    N *= (uint64_t)s->dims[k];
    if (N >= (1ull << 31)) return false;
    si.dims[k] = (uint32_t)s->dims[k];
  }
  si.N = (uint32_t)N;
  uint32_t st = 1;
  for (int k = si.d - 1; k >= 0; --k) {
    si.stride[k] = st;
    st *= si.dims[k];
  }
  for (int k = 0; k < si.d; ++k) {
    si.fdim[k] = make_fastdiv(si.dims[k]);
    si.fstride[k] = make_fastdiv(si.stride[k]);
  }
  // Head/tail split: at most two modes on each side when possible, the
  // split that best balances rows and columns of the CSR view.
  int hlo = si.d - 2 > 1 ? si.d - 2 : 1, hhi = si.d - 1 < 2 ? si.d - 1 : 2;
  if (hlo > hhi) hlo = hhi = si.d / 2;
  int best = hlo;
  double bestv = 1e300;
  for (int h = hlo; h <= hhi; ++h) {
    double mh = 1;
    for (int k = 0; k < h; ++k) mh *= si.dims[k];
    double v = std::fabs(std::log2(mh) - std::log2((double)N / mh));
    if (v < bestv - 1e-12) {
      bestv = v;
      best = h;
    }
  }
  si.h = best;
  si.MH = 1;
  for (int k = 0; k < si.h; ++k) si.MH *= si.dims[k];
  si.MT = si.N / si.MH;
  si.fMT = make_fastdiv(si.MT);
  // CSC head order: ascending (dim, mode); the largest head mode is innermost.
  for (int k = 0; k < si.h; ++k) si.headperm[k] = k;
  for (int a = 0; a < si.h; ++a)
    for (int b = a + 1; b < si.h; ++b) {
      int ma = si.headperm[a], mb = si.headperm[b];
      if (si.dims[mb] < si.dims[ma] || (si.dims[mb] == si.dims[ma] && mb < ma)) {
        si.headperm[a] = mb;
        si.headperm[b] = ma;
      }
    }
  si.nblk = (si.N + kSampleBlockElems - 1) / kSampleBlockElems;
  si.nwords = si.nblk * kSampleBlockWords;
  si.rb = 64;
  si.nrb = (si.MH + si.rb - 1) / si.rb;
  *out = si;
  return true;
}

SampleLayout sample_layout(const ShapeInfo& si, uint64_t cap) {
  SampleLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.hdr = take(512);
  L.bitmap = take((size_t)si.nwords * 8);
  L.wrank = take(((size_t)si.nwords + 1) * 4);
  L.blkcnt = take(((size_t)si.nblk + 1) * 4);
  L.sumsq_part = take((size_t)si.nblk * 8);
  L.coo_l = take((size_t)cap * 8);
  L.rowptr = take(((size_t)si.MH + 1) * 4);
  L.colptr = take(((size_t)si.MT + 1) * 4);
  L.csc_cnt = take(((size_t)si.MT * si.nrb + 1) * 4);
  L.headrow = take((size_t)si.MH * 4);
  L.coo_t = take((size_t)cap * 8);
  L.scan_tmp = take(((size_t)si.MT * si.nrb / 4096 + si.nblk / 4096 + 2) * 4);
  L.cscpos = take((size_t)cap * 4);
  L.headpos = take((size_t)si.MH * 4);
  L.total = o;
  return L;
}

}  // namespace mach

using namespace mach;

extern "C" {

size_t mach_sample_workspace_bytes(const mach_shape* s, uint64_t nnz_cap) {
  ShapeInfo si;
  if (!make_shape_info(s, &si) || nnz_cap < 1 || nnz_cap > (1ull << 31)) return 0;
  return sample_layout(si, nnz_cap).total;
}

uint64_t mach_nnz_capacity(const mach_shape* s, double p) {
  ShapeInfo si;
  if (!make_shape_info(s, &si) || !(p > 0.0 && p <= 1.0)) return 0;
  double N = si.N;
  double c = std::ceil(p * N + 8.0 * std::sqrt(N * p * (1.0 - p))) + 256.0;
  if (c > N) c = N;
  return (uint64_t)c;
}

mach_status mach_layout_info(const mach_shape* s, int32_t* h_out, int32_t* headperm_out) {
  ShapeInfo si;
  if (!make_shape_info(s, &si)) return MACH_EINVAL;
  if (h_out) *h_out = si.h;
  if (headperm_out)
    for (int k = 0; k < si.h; ++k) headperm_out[k] = si.headperm[k];
  return MACH_OK;
}

mach_status mach_sample_offsets(const mach_shape* s, uint64_t nnz_cap, uint64_t* offsets_out,
                                int32_t n) {
  ShapeInfo si;
  if (!make_shape_info(s, &si) || !offsets_out || nnz_cap < 1) return MACH_EINVAL;
  SampleLayout L = sample_layout(si, nnz_cap);
  uint64_t v[6] = {L.coo_l, L.rowptr, L.coo_t, L.colptr, L.bitmap, L.wrank};
  for (int i = 0; i < n && i < 6; ++i) offsets_out[i] = v[i];
  return MACH_OK;
}

mach_status mach_sample(const mach_shape* s, mach_dtype x_dtype, const void* X_dev, double p,
                        uint64_t seed, uint64_t window_id, void* ws, size_t ws_bytes,
                        uint64_t nnz_cap, void* stream) {
  ShapeInfo si;
  if (!make_shape_info(s, &si)) return MACH_EINVAL;
  if (x_dtype != MACH_F64 && x_dtype != MACH_F32) return MACH_EUNSUPPORTED;
  if (!X_dev || !ws || !(p > 0.0 && p <= 1.0)) return MACH_EINVAL;
  if (((uintptr_t)X_dev & 15) || ((uintptr_t)ws & 255)) return MACH_EINVAL;
  if (nnz_cap < 1 || nnz_cap > (1ull << 31)) return MACH_EINVAL;
  SampleLayout L = sample_layout(si, nnz_cap);
  if (ws_bytes < L.total) return MACH_ENOMEM;
  hipError_t e = launch_sample(si, x_dtype == MACH_F64, X_dev, p, seed, window_id, (char*)ws, L,
                               nnz_cap, (hipStream_t)stream);
  return e == hipSuccess ? MACH_OK : MACH_EDEVICE;
}

mach_status mach_sample_ticks(const mach_shape* s, mach_dtype x_dtype, const void* X_dev, double p,
                              uint64_t seed, uint64_t tick0, void* ws, size_t ws_bytes,
                              uint64_t nnz_cap, void* stream) {
  ShapeInfo si;
  if (!make_shape_info(s, &si)) return MACH_EINVAL;
  if (x_dtype != MACH_F64 && x_dtype != MACH_F32) return MACH_EUNSUPPORTED;
  if (!X_dev || !ws || !(p > 0.0 && p <= 1.0)) return MACH_EINVAL;
  if (((uintptr_t)X_dev & 15) || ((uintptr_t)ws & 255)) return MACH_EINVAL;
  if (nnz_cap < 1 || nnz_cap > (1ull << 31)) return MACH_EINVAL;
  if (tick0 > ~0ull - si.dims[si.d - 1]) return MACH_EINVAL;   // ticks must not wrap
  SampleLayout L = sample_layout(si, nnz_cap);
  if (ws_bytes < L.total) return MACH_ENOMEM;
  hipError_t e = launch_sample(si, x_dtype == MACH_F64, X_dev, p, seed, tick0, (char*)ws, L, nnz_cap,
                               (hipStream_t)stream, 1);
  return e == hipSuccess ? MACH_OK : MACH_EDEVICE;
}

mach_status mach_sample_ticks_slide(const mach_shape* s, mach_dtype x_dtype, const void* X_dev,
                                    double p, uint64_t seed, uint64_t tick0, const void* ws_prev,
                                    void* ws, size_t ws_bytes, uint64_t nnz_cap, void* stream) {
  ShapeInfo si;
  if (!make_shape_info(s, &si)) return MACH_EINVAL;
  if (x_dtype != MACH_F64 && x_dtype != MACH_F32) return MACH_EUNSUPPORTED;
  if (!X_dev || !ws || !ws_prev || ws_prev == ws || !(p > 0.0 && p <= 1.0)) return MACH_EINVAL;
  if (((uintptr_t)X_dev & 15) || ((uintptr_t)ws & 255) || ((uintptr_t)ws_prev & 255)) return MACH_EINVAL;
  if (nnz_cap < 1 || nnz_cap > (1ull << 31)) return MACH_EINVAL;
  if (tick0 > ~0ull - si.dims[si.d - 1]) return MACH_EINVAL;
  SampleLayout L = sample_layout(si, nnz_cap);
  if (ws_bytes < L.total) return MACH_ENOMEM;
  hipError_t e = launch_sample_slide(si, x_dtype == MACH_F64, X_dev, p, seed, tick0, (char*)ws, L, nnz_cap,
                                     (const char*)ws_prev, (hipStream_t)stream);
  return e == hipSuccess ? MACH_OK : MACH_EDEVICE;
}

mach_status mach_read_status(const void* ws_sample, const void* ws_solver, void* stream,
                             int32_t* status_out, uint64_t* nnz_out, double* sumsq_out) {
  if (!ws_sample) return MACH_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MACH_EDEVICE;
  SampleHdr h;
  if (hipMemcpy(&h, ws_sample, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return MACH_EDEVICE;
  if (h.magic != kSampleMagic) return MACH_EINVAL;
  int32_t st = h.status;
  if (st == 0 && ws_solver) {
    int32_t s2 = 0;
    if (hipMemcpy(&s2, ws_solver, sizeof(s2), hipMemcpyDeviceToHost) != hipSuccess)
      return MACH_EDEVICE;
    st = s2;
  }
  if (status_out) *status_out = st;
  if (nnz_out) *nnz_out = h.nnz;
  if (sumsq_out) *sumsq_out = h.sumsq;
  return MACH_OK;
}

const char* mach_status_string(mach_status st) {
  switch (st) {
    case MACH_OK: return "ok";
    case MACH_EINVAL: return "invalid argument";
    case MACH_ENOMEM: return "workspace too small or kept count above capacity";
    case MACH_EDEVICE: return "HIP runtime error";
    case MACH_EUNSUPPORTED: return "unsupported input";
    case MACH_EDEGENERATE: return "Gram matrix rank below the requested rank";
    case MACH_ENOCONV: return "eigensolver did not converge";
    default: return "unknown status";
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Solver side
// ---------------------------------------------------------------------------
namespace mach {

bool make_solver_layout(const ShapeInfo& si, const int32_t* ranks, SolverLayout* out) {
  if (!ranks || si.d > 4) return false;
  SolverLayout S;
  std::memset(&S, 0, sizeof(S));
  const int d = si.d, h = si.h;
  // Tucker-n: the last mode may be left uncompressed (rank 0, identity
  // factor) when it is the only tail mode; its "rank" is then its size.
  const int ident = ranks[d - 1] == 0;
  if (ident && d - h != 1) return false;
  S.ident_last = ident;
  auto Reff = [&](int k) -> uint32_t { return (ident && k == d - 1) ? si.dims[k] : (uint32_t)ranks[k]; };
  uint64_t prodR = 1;
  for (int k = 0; k < d; ++k) {
    if (!(ident && k == d - 1) &&
        (ranks[k] < 1 || ranks[k] > kMaxRank || (uint32_t)ranks[k] > si.dims[k]))
      return false;
    prodR *= (uint64_t)Reff(k);
  }
  S.KT = 1;
  S.KH = 1;
  for (int k = 0; k < d; ++k) (k < h ? S.KH : S.KT) *= Reff(k);
  uint32_t smax_sweep = 1, zrows = kBlock, imax = 1, hs_iside_max = 1;
  size_t gmax = 1;
  for (int k = 0; k < d; ++k) {
    ModePlan& m = S.mp[k];
    m.I = si.dims[k];
    m.R = Reff(k);
    if (prodR / m.R >= (1ull << 31)) return false;
    m.K = (uint32_t)(prodR / m.R);
    if (ident && k == d - 1) {     // not updated: no Gram, no eigen state, no HOSVD
      m.kside = 0;
      m.s = 0;
      m.contract_mode = -1;
      S.hosvd_s[k] = 0;
      continue;
    }
    m.kside = m.K < m.I;
    // the column-side warm start maps eigenbases through the other modes'
    // factors, which an identity mode does not have
    if (ident && m.kside) return false;
    m.s = m.kside ? m.K : m.I;
    if (m.R > m.s) return false;
    if (m.kside && m.I > 262144) return false;
    m.contract_mode = -1;
    if (m.s > smax_sweep) smax_sweep = m.s;
    if (m.s > (uint32_t)kSmallEig && m.s > zrows) zrows = m.s;
    if (m.I > imax) imax = m.I;
    gmax = std::max(gmax, (size_t)m.s * m.s);
    uint32_t J = si.N / m.I;
    S.hosvd_kside[k] = m.I > J;
    S.hosvd_s[k] = S.hosvd_kside[k] ? J : m.I;
    if (m.R > S.hosvd_s[k]) return false;
    if (S.hosvd_s[k] > (uint32_t)kSmallEig && S.hosvd_s[k] > zrows) zrows = S.hosvd_s[k];
    if (!S.hosvd_kside[k] && S.hosvd_s[k] > hs_iside_max) hs_iside_max = S.hosvd_s[k];
    // the single tail mode's column-side Gram with more head rows than the
    // sparse Gram holds is never formed
    if (k == d - 1 && h == d - 1 && S.hosvd_kside[k] && si.MH > kSparseGramMaxRows)
      S.hosvd_gram_free = 1;
    else
      gmax = std::max(gmax, (size_t)S.hosvd_s[k] * S.hosvd_s[k]);
  }
  // Views of Y_k (see solver.h).
  const uint32_t* I = si.dims;
  auto R = Reff;
  if (h == 1) {
    S.mp[0].O = 1;
    S.mp[0].Q = S.KT;
  } else {  // h == 2: contract the other head mode
    ModePlan& m0 = S.mp[0];
    m0.contract_mode = 1;
    m0.cO = I[0]; m0.cI = I[1]; m0.cQ = S.KT;
    m0.O = 1; m0.Q = R(1) * S.KT;
    ModePlan& m1 = S.mp[1];
    m1.contract_mode = 0;
    m1.cO = 1; m1.cI = I[0]; m1.cQ = I[1] * S.KT;
    m1.O = R(0); m1.Q = S.KT;
  }
  if (d - h == 1) {
    S.mp[d - 1].O = 1;
    S.mp[d - 1].Q = S.KH;
  } else {  // two tail modes a = h, b = h + 1
    int a = h, b = h + 1;
    ModePlan& ma = S.mp[a];
    ma.contract_mode = b;
    ma.cO = I[a]; ma.cI = I[b]; ma.cQ = S.KH;
    ma.O = 1; ma.Q = R(b) * S.KH;
    ModePlan& mb = S.mp[b];
    mb.contract_mode = a;
    mb.cO = 1; mb.cI = I[a]; mb.cQ = I[b] * S.KH;
    mb.O = R(a); mb.Q = S.KH;
  }
  // Column strides of the other modes in Y_(k): C order over the head modes
  // (KH) and over the tail modes (KT); a contracted second mode of the own
  // side comes first, with stride KT (head side) or KH (tail side).
  {
    uint32_t stH[kMaxD] = {}, stT[kMaxD] = {};
    uint32_t acc = 1;
    for (int j = h - 1; j >= 0; --j) { stH[j] = acc; acc *= R(j); }
    acc = 1;
    for (int j = d - 1; j >= h; --j) { stT[j] = acc; acc *= R(j); }
    for (int k = 0; k < d; ++k) {
      ModePlan& m = S.mp[k];
      const bool head = k < h;
      for (int j = 0; j < d; ++j) {
        if (j == k) continue;
        const bool jhead = j < h;
        if (jhead == head) m.kst[j] = head ? S.KT : S.KH;   // the contracted partner
        else m.kst[j] = jhead ? stH[j] : stT[j];
      }
    }
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  S.status = take(256);
  for (int k = 0; k < d; ++k) S.af[k] = take((size_t)I[k] * 16 * 4);
  for (int k = 0; k < d; ++k) S.af16[k] = take((size_t)I[k] * 16 * 2);
  S.TH = take((size_t)si.MH * S.KT * 4);
  S.TT = take((size_t)si.MT * S.KH * 4);
  if (d - h == 1 && !ident && (size_t)I[d - 1] * 16 * 4 > kTiledFactorBytes) {
    const size_t nt = (I[d - 1] + kTileTicksMin - 1) / kTileTicksMin;
    S.tpart = take(nt * si.MH * 16 * 4);
  }
  for (int k = 0; k < d; ++k) {
    ModePlan& m = S.mp[k];
    if (m.contract_mode >= 0) m.ybuf = take((size_t)m.I * m.K * 4);
    else m.ybuf = k < h ? S.TH : S.TT;
    if (ident && k == d - 1) continue;
    if (m.s <= (uint32_t)kSmallEig) {
      // eigenbasis (s x s), or the I x 16 block of the short-side iteration
      m.V = take(std::max((size_t)m.s * m.s, m.kside ? (size_t)m.I * 16 : 0) * 8);
      m.lam = take((size_t)std::max(m.s, 16u) * 8);
      if (m.kside)
        for (int j = 0; j < d; ++j)
          if (j != k) m.snap[j] = take((size_t)I[j] * 16 * 4);
    } else {
      m.Q64 = take((size_t)m.s * kBlock * 8);
      m.lam = take((size_t)kBlock * 8);
    }
  }
  S.G = take(gmax * 8);
  S.Gpart_elems = std::max<size_t>(std::max<size_t>(64 * (size_t)smax_sweep * smax_sweep,
                                                    16 * (size_t)hs_iside_max * hs_iside_max),
                                   65536);
  // MFMA row-side Grams keep up to 1024 block partials of at most 64 x 64
  if (hs_iside_max > 1) S.Gpart_elems = std::max<size_t>(S.Gpart_elems, 1024 * 64 * 64);
  S.Gpart = take(S.Gpart_elems * 8);
  S.Aw = take((size_t)imax * 16 * 8);
  S.zrows = zrows;
  S.Zs = take((size_t)zrows * kBlock * 8);
  S.Z2s = take((size_t)zrows * kBlock * 8);
  S.Qrs = take((size_t)zrows * kBlock * 8);
  S.Qhs = take((size_t)zrows * kBlock * 8);
  S.H = take(64 * 64 * 8);
  S.VH = take(64 * 64 * 8);
  S.small = take(64 * 64 * 8);
  S.lamH = take(64 * 8);
  S.part = take(64 * 64 * 64 * 8);
  size_t skmax = 1;
  for (int k = 0; k < d; ++k)
    for (uint32_t side : {S.mp[k].s, S.hosvd_s[k]})
      if (side >= 512) skmax = std::max(skmax, (size_t)((side + kSplitK - 1) / kSplitK) * side * 64);
  S.skpart = take(skmax * 8);
  S.pv = take(1024 * 16 * 8);
  S.pi = take(1024 * 16 * 4);
  S.tags = S.status + 16;
  S.sred = take((size_t)kSredElems * 8);
  const size_t gfw_bytes = S.hosvd_gram_free ? (size_t)si.MT * 32 * 8 : 0;
  S.gfw = take(gfw_bytes);
  if (d >= 2) {   // second scratch copy for the last mode's HOSVD
    const size_t sz[18] = {gmax * 8, S.Gpart_elems * 8, (size_t)imax * 16 * 8,
                           (size_t)zrows * kBlock * 8, (size_t)zrows * kBlock * 8,
                           (size_t)zrows * kBlock * 8, (size_t)zrows * kBlock * 8, 64 * 64 * 8,
                           64 * 64 * 8, 64 * 64 * 8, 64 * 8, 64 * 64 * 64 * 8, skmax * 8,
                           1024 * 16 * 8, 1024 * 16 * 4, 256, (size_t)kSredElems * 8, gfw_bytes};
    for (int f = 0; f < 18; ++f) S.laneb[f] = take(sz[f]);
  }
  S.total = o;
  *out = S;
  return true;
}

SolverLayout solver_lane_b(const SolverLayout& S) {
  SolverLayout B = S;
  size_t* f[18] = {&B.G,     &B.Gpart, &B.Aw, &B.Zs,     &B.Z2s, &B.Qrs, &B.Qhs,  &B.H,    &B.VH,
                   &B.small, &B.lamH,  &B.part, &B.skpart, &B.pv,  &B.pi,  &B.tags, &B.sred, &B.gfw};
  for (int i = 0; i < 18; ++i) *f[i] = S.laneb[i];
  return B;
}

SparsePtrs sparse_ptrs(const char* ws, const SampleLayout& L) {
  SparsePtrs p;
  p.hdr = (const SampleHdr*)(ws + L.hdr);
  p.bitmap = (const uint64_t*)(ws + L.bitmap);
  p.wrank = (const uint32_t*)(ws + L.wrank);
  p.coo_l = (const Entry*)(ws + L.coo_l);
  p.coo_t = (const Entry*)(ws + L.coo_t);
  p.rowptr = (const uint32_t*)(ws + L.rowptr);
  p.colptr = (const uint32_t*)(ws + L.colptr);
  p.csc_cnt = (const uint32_t*)(ws + L.csc_cnt);
  p.cscpos = (const uint32_t*)(ws + L.cscpos);
  p.headpos = (const uint32_t*)(ws + L.headpos);
  return p;
}

namespace {

// Kernel timing hook state (host side, not thread safe).
struct TimingPool {
  int every = 0;                         // 0: off; n: one pass of each kind in every n
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
  size_t used[2] = {0, 0};
  uint64_t seen[2] = {0, 0};
};
TimingPool g_timing;

}  // namespace

bool timing_events(int which, hipEvent_t* e0, hipEvent_t* e1) {
  if (g_timing.every <= 0 || which < 0 || which > 1) return false;
  if (g_timing.seen[which]++ % (uint64_t)g_timing.every != 0) return false;
  auto& v = g_timing.ev[which];
  size_t& u = g_timing.used[which];
  if (u == v.size()) {
    // timing only: no system-scope fence (no cache writeback) at each record
    hipEvent_t a, b;
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
      (void)hipEventDestroy(a);
      return false;
    }
    v.push_back({a, b});
  }
  *e0 = v[u].first;
  *e1 = v[u].second;
  ++u;
  return true;
}

namespace {

struct Prepared {
  ShapeInfo si;
  SampleLayout L;
  SolverLayout SL;
  SparsePtrs sp;
};

mach_status prepare(const void* ws_sample, uint64_t cap, const mach_shape* s, const int32_t* ranks,
                    double* const* A, void* ws, size_t ws_bytes, Prepared* P) {
  if (!ws_sample || !ws || !A || !ranks) return MACH_EINVAL;
  if (!make_shape_info(s, &P->si)) return MACH_EINVAL;
  if (P->si.d > 4) return MACH_EUNSUPPORTED;
  if (cap < 1 || cap > (1ull << 31)) return MACH_EINVAL;
  if (!make_solver_layout(P->si, ranks, &P->SL)) return MACH_EINVAL;
  if (ws_bytes < P->SL.total) return MACH_ENOMEM;
  if (((uintptr_t)ws & 255) || ((uintptr_t)ws_sample & 255)) return MACH_EINVAL;
  for (int k = 0; k < P->si.d; ++k)
    if (!A[k] && !(P->SL.ident_last && k == P->si.d - 1)) return MACH_EINVAL;
  P->L = sample_layout(P->si, cap);
  P->sp = sparse_ptrs((const char*)ws_sample, P->L);
  return MACH_OK;
}

}  // namespace
}  // namespace mach

namespace {

// Auxiliary stream and fork/join events per (device, caller stream),
// created on first use and kept for the life of the process.  Streams are
// non-blocking at the default priority.
struct AuxLane {
  int dev;
  hipStream_t caller, st;
  hipEvent_t fork, join;
};
std::mutex g_aux_mu;
std::vector<AuxLane*> g_aux;

AuxLane* aux_lane(hipStream_t caller) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  for (AuxLane* a : g_aux)
    if (a->dev == dev && a->caller == caller) return a;
  AuxLane* a = new AuxLane{dev, caller, nullptr, nullptr, nullptr};
  if (hipStreamCreateWithFlags(&a->st, hipStreamNonBlocking) != hipSuccess) {
    delete a;
    return nullptr;
  }
  if (hipEventCreateWithFlags(&a->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a->join, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(a->st);
    delete a;
    return nullptr;
  }
  g_aux.push_back(a);
  return a;
}

}  // namespace

extern "C" {

size_t mach_solver_workspace_bytes(const mach_shape* s, const int32_t* ranks, mach_dtype prec,
                                   uint64_t nnz_cap) {
  ShapeInfo si;
  SolverLayout SL;
  (void)nnz_cap;
  if (prec != MACH_F32 && prec != MACH_BF16 && prec != MACH_FP8E4M3) return 0;
  if (!make_shape_info(s, &si) || si.d > 4 || !make_solver_layout(si, ranks, &SL)) return 0;
  return SL.total;
}

mach_status mach_solver_reset(const mach_shape* s, const int32_t* ranks, void* ws, size_t ws_bytes,
                              void* stream) {
  ShapeInfo si;
  SolverLayout SL;
  if (!ws || !make_shape_info(s, &si) || si.d > 4 || !make_solver_layout(si, ranks, &SL))
    return MACH_EINVAL;
  if (ws_bytes < SL.total) return MACH_ENOMEM;
  return launch_solver_init(SL, (char*)ws, (hipStream_t)stream) == hipSuccess ? MACH_OK
                                                                             : MACH_EDEVICE;
}

mach_status mach_hosvd(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                       const int32_t* ranks, double* const* A_dev, void* ws, size_t ws_bytes,
                       void* stream) {
  Prepared P;
  mach_status rc = prepare(ws_sample, nnz_cap, s, ranks, A_dev, ws, ws_bytes, &P);
  if (rc != MACH_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  if (launch_solver_init(P.SL, w, st) != hipSuccess) return MACH_EDEVICE;
  // modes with factors (an uncompressed last mode has none)
  const int d = P.SL.ident_last ? P.si.d - 1 : P.si.d;
  // The modes' HOSVDs are independent: the last one (usually the largest
  // Gram) runs on an auxiliary stream with its own scratch, forked from and
  // joined back into `st` by events, beside the others on `st`.
  AuxLane* aux = d >= 2 && P.SL.laneb[0] ? aux_lane(st) : nullptr;
  if (aux && (hipEventRecord(aux->fork, st) != hipSuccess ||
              hipStreamWaitEvent(aux->st, aux->fork, 0) != hipSuccess))
    return MACH_EDEVICE;
  if (aux) {
    const SolverLayout SB = solver_lane_b(P.SL);
    if (launch_hosvd_mode(P.si, P.sp, SB, w, d - 1, ranks[d - 1], A_dev[d - 1], aux->st) != hipSuccess ||
        hipEventRecord(aux->join, aux->st) != hipSuccess)
      return MACH_EDEVICE;
  }
  for (int n = 0; n < (aux ? d - 1 : d); ++n)
    if (launch_hosvd_mode(P.si, P.sp, P.SL, w, n, ranks[n], A_dev[n], st) != hipSuccess)
      return MACH_EDEVICE;
  if (aux && hipStreamWaitEvent(st, aux->join, 0) != hipSuccess) return MACH_EDEVICE;
  return MACH_OK;
}

mach_status mach_hooi_sweep(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                            const int32_t* ranks, double* const* A_dev, mach_dtype prec,
                            int32_t first_mode, void* ws, size_t ws_bytes, double* fit_dev,
                            void* stream) {
  if (prec != MACH_F32 && prec != MACH_BF16 && prec != MACH_FP8E4M3) return MACH_EUNSUPPORTED;
  // mixed precision: bfloat16 factor entries in the sparse passes (both
  // variants); the Gram's inputs in bfloat16 or e4m3
  const int bf16 = prec != MACH_F32;
  Prepared P;
  mach_status rc = prepare(ws_sample, nnz_cap, s, ranks, A_dev, ws, ws_bytes, &P);
  if (rc != MACH_OK) return rc;
  // the last mode updated: an uncompressed last mode keeps its identity
  const int last = P.SL.ident_last ? P.si.d - 2 : P.si.d - 1;
  if (first_mode < 0 || first_mode > last) return MACH_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const int d = last + 1, h = P.si.h;
  const double density = (double)nnz_cap / (double)P.si.N;
  const SampleHdr* hdr = P.sp.hdr;
  bool ok = launch_factors_to_f32(P.si, P.SL, w, A_dev, ranks, hdr, st) == hipSuccess;
  int tail0 = first_mode;
  if (first_mode < h) {
    ok = ok && launch_contract_tail(P.si, P.sp, P.SL, w, ranks, density, bf16, st) == hipSuccess;
    for (int k = first_mode; k < h && ok; ++k) {
      ok = launch_form_y(P.si, P.SL, w, k, hdr, st) == hipSuccess;
      ok = ok && launch_mode_update(P.si, P.SL, w, k, A_dev[k], prec, hdr, st) == hipSuccess;
    }
    tail0 = h;
  }
  if (tail0 < d)
    ok = ok && launch_contract_head(P.si, P.sp, P.SL, w, ranks, density, bf16, st) == hipSuccess;
  for (int k = tail0; k < d && ok; ++k) {
    ok = launch_form_y(P.si, P.SL, w, k, hdr, st) == hipSuccess;
    ok = ok && launch_mode_update(P.si, P.SL, w, k, A_dev[k], prec, hdr, st) == hipSuccess;
  }
  if (ok && fit_dev) ok = launch_fit(P.SL, w, last, hdr, fit_dev, st) == hipSuccess;
  return ok ? MACH_OK : MACH_EDEVICE;
}

mach_status mach_core(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                      const int32_t* ranks, double* const* A_dev, double* G_dev,
                      double* core_norm2_dev, void* ws, size_t ws_bytes, void* stream) {
  Prepared P;
  mach_status rc = prepare(ws_sample, nnz_cap, s, ranks, A_dev, ws, ws_bytes, &P);
  if (rc != MACH_OK) return rc;
  if (!G_dev) return MACH_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const double density = (double)nnz_cap / (double)P.si.N;
  const SampleHdr* hdr = P.sp.hdr;
  bool ok = launch_factors_to_f32(P.si, P.SL, w, A_dev, ranks, hdr, st) == hipSuccess;
  ok = ok && launch_contract_head(P.si, P.sp, P.SL, w, ranks, density, 0, st) == hipSuccess;
  ok = ok && launch_form_y(P.si, P.SL, w, P.si.d - 1, hdr, st) == hipSuccess;
  ok = ok && launch_core(P.si, P.SL, w, A_dev[P.si.d - 1], G_dev, core_norm2_dev, hdr, st) ==
                 hipSuccess;
  return ok ? MACH_OK : MACH_EDEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free core: the scratch of mach_core (status word, float32
// factor copies, the tail-side partial product and the last mode's Y) in a
// fixed device array instead of a caller workspace.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kCoreScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kCoreScratchBytes];

// Device address of `scratch` per device, looked up once per device with
// that device current.  Host code never uses the array's name as an address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// The part of the solver layout that the core's launches touch, packed from
// offset 0: status word and tags, float32 factor copies, TT, and Y of the
// last mode when it is contracted from TT.  Every other offset is 0 and no
// launch of the core reads it.
bool make_core_layout(const ShapeInfo& si, const int32_t* ranks, SolverLayout* out) {
  SolverLayout full;
  if (!make_solver_layout(si, ranks, &full)) return false;
  SolverLayout S;
  std::memset(&S, 0, sizeof(S));
  S.KT = full.KT;
  S.KH = full.KH;
  S.ident_last = full.ident_last;
  for (int k = 0; k < si.d; ++k) {
    S.mp[k] = full.mp[k];
    S.mp[k].ybuf = S.mp[k].V = S.mp[k].lam = S.mp[k].Q64 = 0;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  S.status = take(256);
  S.tags = S.status + 16;
  for (int k = 0; k < si.d; ++k) S.af[k] = take((size_t)si.dims[k] * 16 * 4);
  S.TT = take((size_t)si.MT * S.KH * 4);
  ModePlan& m = S.mp[si.d - 1];
  m.ybuf = m.contract_mode >= 0 ? take((size_t)m.I * m.K * 4) : S.TT;
  S.total = o;
  *out = S;
  return true;
}

}  // namespace

extern "C" {

mach_status mach_core_noalloc(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                              const int32_t* ranks, double* const* A_dev, double* G_dev,
                              double* core_norm2_dev, void* stream) {
  if (!ws_sample || !A_dev || !ranks || !G_dev) return MACH_EINVAL;
  ShapeInfo si;
  if (!make_shape_info(s, &si)) return MACH_EINVAL;
  if (si.d > 4) return MACH_EUNSUPPORTED;
  if (nnz_cap < 1 || nnz_cap > (1ull << 31)) return MACH_EINVAL;
  if ((uintptr_t)ws_sample & 255) return MACH_EINVAL;
  SolverLayout SL;
  if (!make_core_layout(si, ranks, &SL)) return MACH_EINVAL;
  for (int k = 0; k < si.d; ++k)
    if (!A_dev[k] && !(SL.ident_last && k == si.d - 1)) return MACH_EINVAL;
  if (SL.total > kCoreScratchBytes) return MACH_ENOMEM;
  char* w = (char*)scratch_ptr();
  if (!w) return MACH_EDEVICE;
  const SampleLayout L = sample_layout(si, nnz_cap);
  const SparsePtrs sp = sparse_ptrs((const char*)ws_sample, L);
  hipStream_t st = (hipStream_t)stream;
  const double density = (double)nnz_cap / (double)si.N;
  // The status word left by the previous call is cleared by a fill kernel
  // (the sequence stays capturable: no memset node).
  bool ok = launch_solver_init(SL, w, st) == hipSuccess;
  ok = ok && launch_factors_to_f32(si, SL, w, A_dev, ranks, sp.hdr, st) == hipSuccess;
  ok = ok && launch_contract_head(si, sp, SL, w, ranks, density, 0, st) == hipSuccess;
  ok = ok && launch_form_y(si, SL, w, si.d - 1, sp.hdr, st) == hipSuccess;
  ok = ok && launch_core(si, SL, w, A_dev[si.d - 1], G_dev, core_norm2_dev, sp.hdr, st) ==
                 hipSuccess;
  return ok ? MACH_OK : MACH_EDEVICE;
}

mach_status mach_timing_enable(int32_t every) {
  if (every < 0) return MACH_EINVAL;
  g_timing.every = every;
  g_timing.used[0] = g_timing.used[1] = 0;
  g_timing.seen[0] = g_timing.seen[1] = 0;
  return MACH_OK;
}

mach_status mach_timing_read(int32_t which, double* total_ms, int32_t* count) {
  if (which < 0 || which > 1 || !total_ms || !count) return MACH_EINVAL;
  double tot = 0.0;
  for (size_t i = 0; i < g_timing.used[which]; ++i) {
    auto& pr = g_timing.ev[which][i];
    if (hipEventSynchronize(pr.second) != hipSuccess) return MACH_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return MACH_EDEVICE;
    tot += ms;
  }
  *total_ms = tot;
  *count = (int32_t)g_timing.used[which];
  return MACH_OK;
}

int32_t mach_host_selftest(void) {
  // 1. fast division against the hardware divide
  uint64_t x = 88172645463325252ull;
  auto rnd = [&]() {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
  };
  const uint32_t fixed[] = {1u, 2u, 3u, 5u, 7u, 16u, 48u, 64u, 100u, 1440u, 16384u, 262144u,
                            0x7fffffffu, 0x80000000u, 0xffffffffu};
  for (uint32_t d : fixed) {
    FastDiv f = make_fastdiv(d);
    const uint32_t ns[] = {0u, 1u, d - 1, d, d + 1, 0x7fffffffu, 0xfffffffeu, 0xffffffffu};
    for (uint32_t n : ns)
      if (f.div(n) != n / d || f.mod(n) != n % d) return 1;
    for (int t = 0; t < 2000; ++t) {
      uint32_t n = (uint32_t)rnd();
      if (f.div(n) != n / d) return 1;
    }
  }
  for (int t = 0; t < 20000; ++t) {
    uint32_t d = (uint32_t)(rnd() >> (rnd() % 32));
    if (d == 0) d = 1;
    FastDiv f = make_fastdiv(d);
    uint32_t n = (uint32_t)rnd();
    if (f.div(n) != n / d) return 2;
  }
  // 2. round-robin Jacobi schedule: each round pairs every index once, each
  //    sweep meets every pair once.
  for (int np = 2; np <= 64; np += 2) {
    std::vector<int> seen(np * np, 0);
    for (int r = 0; r < np - 1; ++r) {
      std::vector<int> used(np, 0);
      for (int k = 0; k < np / 2; ++k) {
        int m = np - 1, a, b;
        if (k == 0) { a = r; b = m; } else { a = (r + k) % m; b = (r - k + m) % m; }
        if (a == b || used[a] || used[b]) return 3;
        used[a] = used[b] = 1;
        seen[std::min(a, b) * np + std::max(a, b)]++;
      }
    }
    for (int a = 0; a < np; ++a)
      for (int b = a + 1; b < np; ++b)
        if (seen[a * np + b] != 1) return 4;
  }
  // 3. layouts: aligned, increasing, inside the total
  mach_shape s3{3, 0, {128, 16, 16384}};
  ShapeInfo si;
  if (!make_shape_info(&s3, &si) || si.h != 2 || si.MH != 2048 || si.MT != 16384) return 5;
  if (si.headperm[0] != 1 || si.headperm[1] != 0) return 6;
  SampleLayout L = sample_layout(si, 3500000);
  size_t offs[] = {L.hdr, L.bitmap, L.wrank, L.blkcnt, L.sumsq_part, L.coo_l, L.rowptr,
                   L.colptr, L.csc_cnt, L.headrow, L.coo_t, L.scan_tmp, L.total};
  for (size_t i = 0; i + 1 < sizeof(offs) / sizeof(offs[0]); ++i)
    if ((offs[i] & 255) || offs[i + 1] <= offs[i]) return 7;
  int32_t r3[] = {8, 4, 16};
  SolverLayout SL;
  if (!make_solver_layout(si, r3, &SL)) return 8;
  if (SL.mp[0].s != 64 || !SL.mp[0].kside || SL.mp[1].s != 16 || SL.mp[1].kside ||
      SL.mp[2].s != 32 || !SL.mp[2].kside)
    return 9;
  for (int k = 0; k < 3; ++k)
    if (SL.mp[k].O * SL.mp[k].Q != SL.mp[k].K) return 10;
  if (SL.hosvd_s[2] != 2048 || !SL.hosvd_kside[2] || SL.hosvd_s[0] != 128) return 11;
  mach_shape s4{4, 0, {64, 64, 64, 256}};
  int32_t r4[] = {10, 10, 10, 10};
  if (!make_shape_info(&s4, &si) || si.h != 2 || !make_solver_layout(si, r4, &SL)) return 12;
  for (int k = 0; k < 4; ++k)
    if (SL.mp[k].O * SL.mp[k].Q != SL.mp[k].K || SL.mp[k].kside) return 13;
  return 0;
}

}  // extern "C"
