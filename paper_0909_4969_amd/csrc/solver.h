// Solver-side internals: the per-mode tensor views of a HOOI sweep, the
// solver workspace layout and the kernel launchers.
//
// A sweep splits the modes into head modes 0..h-1 and tail modes h..d-1
// (ShapeInfo).  Two sparse passes per sweep serve all d mode updates:
//   TH = Xhat x_{k >= h} A_k^T   (MH x KT, from the CSR copy; KT = prod_{k>=h} R_k)
//   TT = Xhat x_{k <  h} A_k^T   (MT x KH, from the CSC copy; KH = prod_{k<h} R_k)
// TH is formed before the head updates and TT after them, so each Y below
// uses the factors Alg. 2 prescribes (modes updated in order 1..d).  Mode
// products along different modes commute (Section 2.1), so
//   Y_k = TH x_{j in head, j != k} A_j^T   for a head mode k,
//   Y_k = TT x_{j in tail, j != k} A_j^T   for a tail mode k,
// which is the tensor of Alg. 2's "Y <-" line with rows permuted.
#pragma once

#include "mach_internal.h"

namespace mach {

// Y_k viewed as a 3-way array (O, I_k, Q), element (o, i, q) at
// (o * I_k + i) * Q + q; the matricization Y_(k) is I_k x (O*Q).
struct YView {
  const float* base;
  uint32_t O, I, Q;
};

struct ModePlan {
  uint32_t I, R, K;        // I_k, R_k, K_k = prod_{j != k} R_j
  uint32_t s;              // Gram side = min(I, K)
  int kside;               // 1: Gram is Y^T Y (K x K); 0: Y Y^T (I x I)
  // dense contraction that forms Y_k from TH/TT (contract == -1: none)
  int contract_mode;       // mode whose factor is applied
  uint32_t cO, cI, cQ;     // view of the source for that contraction
  uint32_t O, Q;           // view of Y_k
  size_t ybuf;             // byte offset of Y_k's buffer (or of TH/TT)
  size_t V, lam, Q64;      // eigen state: V (s x s) or Q64 (s x kBlock)
  // column side, s <= 64: the other modes' float32 factors at the last solve
  // (I_j x 16 each) and the stride of each other mode's column index in Y_(k)
  size_t snap[kMaxD];
  uint32_t kst[kMaxD];
};

constexpr uint32_t kBlock = 64;          // subspace block for sides > kSmallEig
// sred: Gram of a sweep mode (64 x 64), C_j of up to 3 other modes (3 x 256),
// 16 x 16 Gram of a tall factor
constexpr uint32_t kSredGram = 0, kSredCtc = 4096, kSredTall = 4096 + 768, kSredElems = 4096 + 768 + 256;
// Column-side Gram of the single tail mode from the sparse layouts: at most
// this many head rows (one float64 accumulator row per wave in LDS); beyond
// it the mode's HOSVD runs without forming the Gram.
constexpr uint32_t kSparseGramMaxRows = 2048;
constexpr uint32_t kSplitK = 128;        // summation slice of the split products by G
constexpr uint32_t kMfmaGramMaxRows = 1024;  // row-side HOSVD Grams on MFMA up to this side
// Tiled head-row pass: the tail factor is tiled when its float32 copy (16
// columns) exceeds kTiledFactorBytes; tiles span kTileTicksMin..kTileTicksMax
// ticks.
constexpr uint32_t kTiledFactorBytes = 16384;
constexpr uint32_t kTileTicksMin = 128, kTileTicksMax = 256;

// Status region: int32 status word at +0, int32 tags[16] at +16 (eigen
// warm-start tags of modes 0..7, then kTagRR, kTagCold, kTagDone), int32
// solver statistics at +96 (Jacobi sweeps of the last solve of modes 0..7,
// +1000 if warm-started; subspace-iteration steps of the HOSVD of modes
// 0..7 at +128, +10000 if not converged), doubles from +192.
constexpr int kTagRR = 8, kTagCold = 9, kTagDone = 10, kTagRitz = 11;

struct SolverLayout {
  size_t status;                         // see above
  size_t af[kMaxD];                      // float32 factors, I_k x 16
  size_t af16[kMaxD];                    // bfloat16 copies for the mixed-precision sweep
  size_t TH, TT;
  size_t G, Gpart, Gpart_elems;          // float64 Gram and its partials
  size_t Aw;                             // float64 I_max x 16 scratch
  uint32_t zrows;                        // rows of the subspace scratch blocks
  size_t Zs, Z2s, Qrs, Qhs;              // float64 zrows x 64 each
  size_t H, VH, lamH, small;             // float64 64 x 64 (lamH: 64)
  size_t part;                           // float64 64 x 64 x 64 partials
  size_t skpart;                         // float64 split-K partials of G * block
  size_t pv, pi;                         // column-max partials (1024 x 16)
  size_t tags;                           // int32 tags of warm starts and early exits (16)
  size_t sred;                           // float64 reduced partials (kSredElems)
  size_t gfw;                            // Gram-free tail HOSVD: float64 MT x 32 block (else 0 bytes)
  // Tiled head-row pass (one tail mode whose factor is too large for LDS):
  // float32 partial rows, tiles x MH x 16; 0 when the pass is not tiled.
  size_t tpart;
  // A second copy of the scratch above (G .. gfw), used by the HOSVD of the
  // last mode when it runs on its own stream beside the other modes; 0 when
  // there is none (d == 1).
  size_t laneb[18];
  size_t total;
  int ident_last;                        // the last mode is left uncompressed (Tucker-n)
  ModePlan mp[kMaxD];
  uint32_t KT, KH, hosvd_s[kMaxD];
  int hosvd_kside[kMaxD];
  // The last mode's HOSVD runs without forming its Gram (the single tail
  // mode, column side, more head rows than the sparse Gram holds).
  int hosvd_gram_free;
};

bool make_solver_layout(const ShapeInfo& si, const int32_t* ranks, SolverLayout* out);
// The layout with the second scratch copy in place of the first.
SolverLayout solver_lane_b(const SolverLayout& S);

struct SparsePtrs {
  const SampleHdr* hdr;
  const uint64_t* bitmap;
  const uint32_t* wrank;
  const Entry* coo_l;
  const Entry* coo_t;
  const uint32_t* rowptr;
  const uint32_t* colptr;
  const uint32_t* csc_cnt;
  const uint32_t* cscpos;   // CSC position of each CSR (l-ordered) entry
  const uint32_t* headpos;  // position of each head row in the CSC head order
};

SparsePtrs sparse_ptrs(const char* ws_sample, const SampleLayout& L);

// ---- launchers -------------------------------------------------------------
// Sparse passes (ttm.hip).  density = nnz_cap / N, used only to pick the
// number of lanes per segment.
hipError_t launch_contract_tail(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                char* ws, const int32_t* ranks, double density, int bf16,
                                hipStream_t st);
hipError_t launch_contract_head(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                char* ws, const int32_t* ranks, double density, int bf16,
                                hipStream_t st);
hipError_t launch_form_y(const ShapeInfo& si, const SolverLayout& SL, char* ws, int k,
                         const SampleHdr* hdr, hipStream_t st);
hipError_t launch_factors_to_f32(const ShapeInfo& si, const SolverLayout& SL, char* ws,
                                 double* const* A, const int32_t* ranks, const SampleHdr* hdr,
                                 hipStream_t st);

// Gram, eigensolve and factor update of one mode from Y_k (gram.hip, eig.hip).
// prec: input precision of the sweep Gram (MACH_F32, MACH_BF16 or
// MACH_FP8E4M3), float32 accumulation.
hipError_t launch_mode_update(const ShapeInfo& si, const SolverLayout& SL, char* ws, int k,
                              double* A_out, int prec, const SampleHdr* hdr, hipStream_t st);
hipError_t launch_fit(const SolverLayout& SL, char* ws, int k, const SampleHdr* hdr, double* fit,
                      hipStream_t st);
hipError_t launch_core(const ShapeInfo& si, const SolverLayout& SL, char* ws, const double* A_last,
                       double* G, double* norm2, const SampleHdr* hdr, hipStream_t st);
hipError_t launch_hosvd_mode(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                             char* ws, int n, int R, double* A_out, hipStream_t st);
hipError_t launch_solver_init(const SolverLayout& SL, char* ws, hipStream_t st);

// Kernel timing hook (api.hip): while enabled, the sparse passes are
// launched with start/stop events taken from a pool; which = 0 for the
// pass over head rows, 1 for the pass over tail columns.
bool timing_events(int which, hipEvent_t* e0, hipEvent_t* e1);

}  // namespace mach
