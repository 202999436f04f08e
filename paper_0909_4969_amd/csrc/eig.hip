// Float64 top-R eigensolve of a Gram matrix and the factor update it
// feeds (Alg. 1 HOSVD loop and Alg. 2 inner loop: "A <- r leading left
// singular vectors"; Section 2.2 on the SVD), plus the fit and the core
// (eq. eqcore, the last line of Alg. 1/2) with its norm (eq. norm).
//
// Sides up to 64: one workgroup runs cyclic two-sided Jacobi (Golub & Van
// Loan, "Matrix Computations", Sec. 8.5) on the whole matrix in LDS with
// the round-robin parallel ordering, optionally warm-started from the
// previous eigenvector matrix of the same mode (W = V^T G V is close to
// diagonal once HOOI settles, and Jacobi converges quadratically).
// Larger sides: block subspace iteration with float64 CholeskyQR2
// orthonormalisation and Rayleigh-Ritz on a 64-column block (the projected
// 64 x 64 problem goes to the Jacobi kernel), until the residuals of the
// top R Ritz pairs fall below 1e-12 of the largest.
//
// The factor of a row-side Gram is its top-R eigenvectors.  For a
// column-side Gram of M (rows i, columns j) it is M v / sqrt(lambda),
// orthonormalised again by CholeskyQR2 in float64.  Every factor then gets
// the sign rule: in each column the entry of largest magnitude is positive
// (lowest row on ties).
#include <cmath>

#include <algorithm>

#include "solver.h"

namespace mach {

hipError_t launch_gram_y(const SolverLayout& SL, char* ws, int k, int prec, const SampleHdr* hdr,
                         hipStream_t st);
hipError_t launch_gram_y_partials(const SolverLayout& SL, char* ws, int k, int prec,
                                  const SampleHdr* hdr, hipStream_t st, uint32_t* nchunk);
hipError_t launch_gram_xhat(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                            char* ws, int n, hipStream_t st);
bool sparse_tail_gram_ok(const ShapeInfo& si, const SolverLayout& SL, int n);
hipError_t launch_gram_tail_sparse(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                                   char* ws, hipStream_t st);

namespace {

constexpr int kMaxSweeps = 40;
// Jacobi stops when the off-diagonal Frobenius norm of the leading rows is
// below 1e-8 of their diagonal's: the eigenvectors are then exact for a
// matrix within 1e-8 (relative) of the Gram, whose own float32 rounding is
// about 1e-7, so a tighter test would only resolve rounding noise.
constexpr double kOffTol2 = 1e-16;

// Stopping tolerances of a sweep's eigensolve, matched to the precision of
// its input: with float32 TTM and Gram inputs, off-diagonal mass below 1e-16
// of the diagonal mass (Jacobi) and Ritz residuals below 1e-10 of theta_1
// (block and subspace iterations; above 1e-8 at the end is a failure); with
// bfloat16 or e4m3 inputs, whose rounding perturbs the Gram by about 1e-3 of
// its norm or more, 1e-12 and 1e-6 (1e-4): the eigensolve's own error stays
// a thousand times below its input's.
struct SolveTol {
  double off2, res, res_fail;
};
__host__ __device__ inline SolveTol solve_tol(int prec) {
  return prec == MACH_F32 ? SolveTol{kOffTol2, 1e-10, 1e-8} : SolveTol{1e-12, 1e-6, 1e-4};
}

// Round-robin pairing of NP indices (NP even): in round r < NP - 1, pair k
// joins (r + k) mod (NP - 1) and (r - k) mod (NP - 1), and pair 0 joins r
// and NP - 1; every pair of indices meets exactly once per sweep.
template <int NP>
__device__ __forceinline__ void jpair_c(int r, int k, int* p, int* q) {
  constexpr int m = NP - 1;
  int a = (r + k) % m, b = (r - k + m) % m;
  if (k == 0) {
    a = r;
    b = m;
  }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

struct Status {
  const SampleHdr* hdr;
  int32_t* st;        // solver status word
  const int32_t* done;  // optional early-exit flag (converged); may be null
  __device__ __forceinline__ bool skip() const {
    return hdr->status != 0 || *st != 0 || (done && *done);
  }
};

__device__ void block_sum2(double& a, double& b, double (*red)[4]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  a = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
  b = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  __syncthreads();
}

struct JacArgs {
  const double* G;     // n x n symmetric: entry (x, y) = sum_c G[(x * n + y) * nchunk + c]
  uint32_t nchunk;
  uint32_t n;
  double* V;           // in: warm start if tagval != 0 and *tag == tagval; out: eigenvectors (columns, sorted)
  double* lam;         // out: eigenvalues, descending
  int32_t* tag;
  int32_t tagval;
  int rtop;            // leading eigenpairs that must converge
  double tol2;         // stopping threshold on off-diagonal / diagonal mass
  Status s;
};

// LDS state of the Jacobi kernels for a padded size NP (power of two).
// Broadcast of a float64 register from lane `src` (wave-uniform) to the wave.
__device__ inline double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Right-looking Cholesky of a 16 x 16 symmetric positive definite block held
// by rows in registers: lane x < 16 passes row x in a[], and gets back row x
// of L (zeros above the diagonal).  Only entries on and below the diagonal
// are read; a pivot below 1e-300 is replaced by 1 (degenerate input stays
// finite; the eigenvalue test reports it).  Every lane of the wave calls it:
// the column of L is broadcast from lanes 0..15 with readlane.
__device__ inline void chol16_wave(double (&a)[16], int x) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double d = lane_bcast(a[j], j);
    const double sd = d > 1e-300 ? sqrt(d) : 1.0;
    const double l = x == j ? sd : a[j] / sd;
    a[j] = l;
#pragma unroll
    for (int k = j + 1; k < 16; ++k) a[k] = fma(-l, lane_bcast(l, k), a[k]);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k > x) a[k] = 0.0;
}

template <int NP>
struct JacLds {
  double A[NP][NP + 1];                 // the matrix being diagonalised
  double V[NP][NP + 1];                 // accumulated rotations
  double W[NP][NP + 1];                 // scratch (warm-start products; second copy of A in Jacobi)
  int rk[NP];
  double red[2][16];
};

// Block-wide sums of two values over NT threads (fixed order).
template <int NT>
__device__ void block_sum2n(double& a, double& b, double (*red)[16]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int i = 0; i < NT / 64; ++i) {
    a += red[0][i];
    b += red[1][i];
  }
  __syncthreads();
}

typedef double v4d __attribute__((ext_vector_type(4)));

// D = op(A) B for NP x NP matrices in LDS (op(A) = A^T when TA) on float64
// MFMA: each wave takes 16 x 16 output tiles and runs
// v_mfma_f64_16x16x4f64 over the inner index in steps of 4 (operand lane
// l: row / column l % 16, inner index l / 16; result register v of lane l:
// row l / 16 + 4 v, column l % 16).  D may alias A or B (every read
// completes before the first write).
template <int NP, int NT, bool TA>
__device__ void lds_gemm(double (*A)[NP + 1], double (*B)[NP + 1], double (*D)[NP + 1]) {
  constexpr int TT = NP / 16, NW = NT / 64, TPW = (TT * TT + NW - 1) / NW;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  v4d acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = w + u * NW;
    acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
    if (t < TT * TT) {
      const int ti = t / TT, tj = t % TT;
      v4d c = acc[u];
#pragma unroll 4
      for (int k0 = 0; k0 < NP; k0 += 4) {
        const double av = TA ? A[k0 + lk][ti * 16 + li] : A[ti * 16 + li][k0 + lk];
        const double bv = B[k0 + lk][tj * 16 + li];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
      }
      acc[u] = c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = w + u * NW;
    if (t < TT * TT) {
      const int ti = t / TT, tj = t % TT;
#pragma unroll
      for (int v = 0; v < 4; ++v) D[ti * 16 + lk + 4 * v][tj * 16 + li] = acc[u][v];
    }
  }
  __syncthreads();
}

// Sets the start basis L.V — the identity, the warm start Vin (n x n
// row-major, when warm), or the one already in L.V (in_lds) — and, unless it
// is the identity, replaces L.A = G by V^T G V.  Expects L.A = G (padded
// with zeros).
// V (NP x NP in LDS) = Vin (n x n row-major) padded with the identity, or
// the identity when !use.  The loads are unconditional, at indices clamped
// into Vin (finite entries), and the padding is set by factors 0 and 1: a
// predicated load, or a select the compiler turns back into one, is a branch
// that waits for its load.
template <int NP, int NT>
__device__ __forceinline__ void load_basis(double (*V)[NP + 1], int n, bool use, const double* Vin) {
  static_assert(NP * NP % NT == 0, "whole entries per thread");
  constexpr int NE = NP * NP / NT;
  const int tid = threadIdx.x;
  double v[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) v[u] = 0.0;
  if (use) {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = u * NT + tid, x = e / NP, y = e % NP;
      v[u] = Vin[min(x, n - 1) * n + min(y, n - 1)];
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = u * NT + tid, x = e / NP, y = e % NP;
    const double m = (use && x < n && y < n) ? 1.0 : 0.0;
    V[x][y] = v[u] * m + (1.0 - m) * (x == y ? 1.0 : 0.0);
  }
}

// A (NP x NP in LDS) = the n x n matrix summed from its chunk partials
// (part[(x n + y) nchunk + c]), zero padded, each entry summed in chunk
// order; loads unconditional at clamped indices, the padding zeroed by a
// factor 0 (as in load_basis).
template <int NP, int NT>
__device__ __forceinline__ void load_gram(double (*A)[NP + 1], int n, const double* part,
                                          uint32_t nchunk) {
  static_assert(NP * NP % NT == 0, "whole entries per thread");
  constexpr int NE = NP * NP / NT;
  const int tid = threadIdx.x;
  double g[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) g[u] = 0.0;
  for (uint32_t c = 0; c < nchunk; ++c) {
    double p[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = u * NT + tid, x = e / NP, y = e % NP;
      p[u] = part[(size_t)(min(x, n - 1) * n + min(y, n - 1)) * nchunk + c];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = u * NT + tid, x = e / NP, y = e % NP;
      g[u] += p[u] * ((x < n && y < n) ? 1.0 : 0.0);
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = u * NT + tid;
    A[e / NP][e % NP] = g[u];
  }
}

template <int NP, int NT>
__device__ void jacobi_setup(JacLds<NP>& L, int n, bool warm, const double* Vin, bool in_lds = false) {
  const int tid = threadIdx.x;
  if (!in_lds) load_basis<NP, NT>(L.V, n, warm, Vin);
  warm = warm || in_lds;
  __syncthreads();
  if (!warm) return;
  // W = G V, then A = V^T W (padding: G zero, V the identity)
  lds_gemm<NP, NT, false>(L.A, L.V, L.W);
  lds_gemm<NP, NT, true>(L.V, L.W, L.A);
  for (int e = tid; e < NP * NP; e += NT) {
    int x = e / NP, y = e % NP;
    if (x < y) {
      double m = 0.5 * (L.A[x][y] + L.A[y][x]);
      L.A[x][y] = m;
      L.A[y][x] = m;
    }
  }
  __syncthreads();
}

// Jacobi rotation of the pair (p, q) of a symmetric matrix (Golub & Van
// Loan, Sec. 8.5, sym.schur2): t = tan of the smaller angle that zeroes
// a_pq, c = cos, s = sin.  t is formed in float32 from the pair scaled by a
// power of two, with hardware reciprocals (its rounding leaves a_pq at
// about 1e-7 of its size, which the next sweeps remove like any other
// off-diagonal entry); c and s follow from t in float64, so the rotation is
// orthogonal to float64 rounding.  The identity when a_pq is negligible
// against the diagonal.  No branches: every lane runs the same instructions.
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double* c, double* s) {
  const bool act = fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * (fabs(app) + fabs(aqq));
  const int e = ilogb(act ? apq : 1.0);
  const float num = (float)ldexp(aqq - app, -e), den = (float)ldexp(2.0 * apq, -e);
  const float th = num * __builtin_amdgcn_rcpf(den);
  const float ath = fabsf(th);
  const float tbig = 0.5f * __builtin_amdgcn_rcpf(th);
  const float tsml = __builtin_amdgcn_rcpf(ath + __builtin_amdgcn_sqrtf(fmaf(th, th, 1.0f)));
  const float t = ath > 1e15f ? tbig : copysignf(tsml, th);
  const double td = act ? (double)t : 0.0;
  const double cc = act ? rsqrt(fma(td, td, 1.0)) : 1.0;
  *c = cc;
  *s = td * cc;
}

// Cyclic two-sided Jacobi on L.A (n x n padded to NP, symmetric),
// accumulating rotations into L.V.  Each round applies the NP/2 disjoint
// rotations of the round-robin ordering.  Thread (ia, ib) of the first
// (NP/2)^2 owns the 2x2 block of rows (p_ia, q_ia) and columns (p_ib, q_ib):
// it reads the block from the current copy of A, writes J_ia^T block J_ib
// into the other copy (L.W), and rotates the same 2x2 block of V in place
// by J_ib (every entry of A and V belongs to exactly one block per round),
// so a round needs one barrier; with NP = 16 the blocks are one wave, whose
// LDS accesses stay in program order, and the rounds need none.  Every
// rotation is computed by the same instructions from the same inputs
// wherever it is used: lane l computes the rotation of pair l mod NP/2 (its
// own column pair) and, for NP <= 32, its row pair's as well; for NP = 64
// the row pair's comes from lane ia of the wave by a shuffle.
//
// Only the leading `rtop` eigenpairs are wanted, so the stopping test looks
// at the rows of the rtop largest diagonal entries: it stops when their
// off-diagonal mass is below tol2 of their diagonal mass.  Returns the
// number of sweeps run; *conv tells whether the test passed.  On return
// L.A holds the rotated matrix; L.W is overwritten.
template <int NP, int NT>
__device__ int jacobi_core(JacLds<NP>& L, int n, int rtop, bool* conv, double tol2 = kOffTol2) {
  constexpr int PAIRS = NP / 2, ROUNDS = NP - 1, NB = PAIRS * PAIRS, NW = NT / 64;
  constexpr bool kOneWave = NB == 64, kLocalRows = NP <= 32;
  static_assert(NB <= NT && NB % 64 == 0 && 64 % PAIRS == 0 && NP <= 64 && NW <= 16,
                "one thread per 2x2 block, whole waves");
  static_assert(ROUNDS % 2 == 1, "an odd number of buffer swaps per sweep");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double (*A)[NP + 1] = L.A;
  double (*B)[NP + 1] = L.W;
  *conv = false;
  int sweep = 0;
  for (; sweep <= kMaxSweeps; ++sweep) {
    // stopping test: wave w takes rows w, w + NW, ...; the rank of a row's
    // diagonal entry (descending, ties by index) is a ballot over the lanes
    {
      const int yl = lane < NP ? lane : 0;
      const double dy = A[yl][yl];
      double acc = 0.0, dgs = 0.0;
      for (int x = w; x < n; x += NW) {
        const double v = A[x][yl], dx = A[x][x];
        const unsigned long long m = __ballot(lane < n && (dy > dx || (dy == dx && lane < x)));
        if (__popcll(m) < (unsigned)rtop) {
          acc = fma(v, lane < n && lane != x ? v : 0.0, acc);
          dgs = fma(dx, dx, dgs);
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) {
        L.red[0][w] = acc;
        L.red[1][w] = dgs;
      }
    }
    __syncthreads();
    if (tid == 0) {
      double off = 0.0, dg = 0.0;
      for (int i = 0; i < NW; ++i) {
        off += L.red[0][i];
        dg += L.red[1][i];
      }
      L.rk[0] = (off <= tol2 * dg) || dg == 0.0;
    }
    __syncthreads();
    *conv = L.rk[0] != 0;
    __syncthreads();
    if (*conv || sweep == kMaxSweeps) break;
    // (no barrier inside a branch that can differ between waves)
    if (!kOneWave || w == 0) {
      for (int r = 0; r < ROUNDS; ++r) {
        if (tid < NB) {
          const int ia = tid / PAIRS, ib = tid % PAIRS;
          int pa, qa, pb, qb;
          jpair_c<NP>(r, ia, &pa, &qa);
          jpair_c<NP>(r, ib, &pb, &qb);
          // everything this thread reads, before anything is written
          const double bpp = A[pb][pb], bqq = A[qb][qb], bpq = A[pb][qb];
          double app = 0.0, aqq = 0.0, apq = 0.0;
          if (kLocalRows) {
            app = A[pa][pa];
            aqq = A[qa][qa];
            apq = A[pa][qa];
          }
          const double w11 = A[pa][pb], w12 = A[pa][qb], w21 = A[qa][pb], w22 = A[qa][qb];
          const double v11 = L.V[pa][pb], v12 = L.V[pa][qb], v21 = L.V[qa][pb], v22 = L.V[qa][qb];
          double cb, sb, ca, sa;
          jacobi_rotation(bpp, bqq, bpq, &cb, &sb);
          if (kLocalRows) {
            jacobi_rotation(app, aqq, apq, &ca, &sa);
          } else {
            ca = __shfl(cb, ia, 64);
            sa = __shfl(sb, ia, 64);
          }
          const double r11 = ca * w11 - sa * w21, r12 = ca * w12 - sa * w22;
          const double r21 = sa * w11 + ca * w21, r22 = sa * w12 + ca * w22;
          B[pa][pb] = cb * r11 - sb * r12;
          B[pa][qb] = sb * r11 + cb * r12;
          B[qa][pb] = cb * r21 - sb * r22;
          B[qa][qb] = sb * r21 + cb * r22;
          L.V[pa][pb] = cb * v11 - sb * v12;
          L.V[pa][qb] = sb * v11 + cb * v12;
          L.V[qa][pb] = cb * v21 - sb * v22;
          L.V[qa][qb] = sb * v21 + cb * v22;
        }
        if (kOneWave) __builtin_amdgcn_wave_barrier();
        else __syncthreads();
        double (*T)[NP + 1] = A;
        A = B;
        B = T;
      }
    }
    if (kOneWave) {
      // sweeps 0..sweep done, ROUNDS (odd) swaps each
      A = (sweep & 1) ? L.A : L.W;
      B = (sweep & 1) ? L.W : L.A;
      __syncthreads();
    }
  }
  // ROUNDS is odd: after an odd number of sweeps the matrix is in L.W
  if (sweep & 1) {
    for (int e = tid; e < NP * NP; e += NT) L.A[e / NP][e % NP] = L.W[e / NP][e % NP];
    __syncthreads();
  }
  return sweep;
}

// Ranks of the eigenvalues (descending, ties by index) into L.rk; writes
// lam[rank] and Vout[row * n + rank] (n x n) when given.
template <int NP, int NT>
__device__ void jacobi_sort_store(JacLds<NP>& L, int n, double* lam, double* Vout) {
  const int tid = threadIdx.x;
  if (tid < n) {
    double lx = L.A[tid][tid];
    int rank = 0;
    for (int y = 0; y < n; ++y) {
      double ly = L.A[y][y];
      rank += (ly > lx) || (ly == lx && y < tid);
    }
    L.rk[tid] = rank;
    if (lam) lam[rank] = lx;
  }
  __syncthreads();
  if (Vout)
    for (int e = tid; e < n * NP; e += NT) {
      int row = e / NP, x = e % NP;
      if (x < n) Vout[row * n + L.rk[x]] = L.V[row][x];
    }
}

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_jacobi_small(JacArgs a) {
  if (a.s.skip()) return;
  __shared__ JacLds<NP> L;
  const int n = (int)a.n, tid = threadIdx.x;
  const bool warm = a.tagval != 0 && *a.tag == a.tagval;
  load_gram<NP, NT>(L.A, n, a.G, a.nchunk);
  __syncthreads();
  jacobi_setup<NP, NT>(L, n, warm, a.V);
  bool conv;
  jacobi_core<NP, NT>(L, n, a.rtop, &conv, a.tol2);
  jacobi_sort_store<NP, NT>(L, n, a.lam, a.V);
  if (tid == 0) {
    if (a.tagval != 0) *a.tag = a.tagval;
    if (!conv) atomicCAS(a.s.st, 0, MACH_ENOCONV);
  }
}

// Column-side warm start.  The eigenvectors of G = Y_(k)^T Y_(k) live in the
// coordinates of the other modes' factor columns (Y_(k) = Xhat_(k) times the
// Kronecker product of the other factors), and those columns rotate from one
// sweep to the next, mostly within groups of nearly equal singular values, so
// the previous eigenbasis V_old is not a good start as it stands.  With
// C_j = A_j,old^T A_j,new (R_j x R_j) for every other mode j, A_j,new ~=
// A_j,old C_j, hence Y_new ~= Y_old P with P = kron_j C_j (in the column
// order of Y_(k)), G_new ~= P^T G_old P, and P^T V_old is the previous
// eigenbasis in the current coordinates.  P is orthogonal up to how far the
// factor subspaces moved; Newton-Schulz steps restore orthogonality.
// part[(slot * 256 + a * 16 + b) * kCtcChunks + chunk] = sum over the chunk's
// rows i of old[i][a] * cur[i][b] (float32 factors I_j x 16, float64 sums).
constexpr uint32_t kCtcChunks = 64;

// Copies of the other modes' float32 factors, taken after a column-side solve.
struct SnapArgs {
  const float4* src[3];
  float4* dst[3];
  uint32_t n4[3];
  int n;
};


struct CtcArgs {
  const float* old[3];
  const float* cur[3];
  uint32_t I[3];
  uint32_t nch[3];        // chunks of slot j: ctc_chunks(I_j)
  int n;
};

__host__ __device__ inline uint32_t ctc_chunks(uint32_t I) {
  uint32_t c = (I + 255) / 256;
  return c < 1 ? 1 : (c > kCtcChunks ? kCtcChunks : c);
}

// Rows are staged through LDS 256 at a time (coalesced float4 loads), then
// thread (a, b) sums old[i][a] * cur[i][b] over them.
__global__ __launch_bounds__(256) void k_ctc_partial(CtcArgs a, double* __restrict__ part, Status s) {
  if (s.skip()) return;
  const int slot = blockIdx.y;
  if (slot >= a.n || blockIdx.x >= a.nch[slot]) return;
  __shared__ float so[256][17];
  __shared__ float sc[256][17];
  const uint32_t I = a.I[slot];
  const uint32_t rows = (I + a.nch[slot] - 1) / a.nch[slot];
  const uint32_t i0 = blockIdx.x * rows, i1 = min(I, i0 + rows);
  const int aa = threadIdx.x >> 4, bb = threadIdx.x & 15;
  const float4* po = reinterpret_cast<const float4*>(a.old[slot]);
  const float4* pc = reinterpret_cast<const float4*>(a.cur[slot]);
  double acc = 0.0;
  for (uint32_t b0 = i0; b0 < i1; b0 += 256) {
    const uint32_t nb = min(256u, i1 - b0);
    for (uint32_t e = threadIdx.x; e < nb * 4; e += 256) {
      const float4 vo = po[(size_t)b0 * 4 + e], vc = pc[(size_t)b0 * 4 + e];
      const uint32_t r = e >> 2, c = (e & 3) * 4;
      so[r][c] = vo.x; so[r][c + 1] = vo.y; so[r][c + 2] = vo.z; so[r][c + 3] = vo.w;
      sc[r][c] = vc.x; sc[r][c + 1] = vc.y; sc[r][c + 2] = vc.z; sc[r][c + 3] = vc.w;
    }
    __syncthreads();
    for (uint32_t r = 0; r < nb; ++r) acc = fma((double)so[r][aa], (double)sc[r][bb], acc);
    __syncthreads();
  }
  part[((size_t)slot * 256 + threadIdx.x) * kCtcChunks + blockIdx.x] = acc;   // chunks < nch[slot] used
}

// Sums of chunked partials, one wave per entry: lane c adds chunks c,
// c + 64, ... of entry e (in[e * es + c * cs]), then a fixed butterfly adds
// the lanes; out[e] gets the total.  Entries come in groups of gsize with
// their own chunk counts nch[e / gsize] (at most 4 groups).  The order of
// the additions is fixed, so the result is reproducible.
struct ReduceArgs {
  const double* in;
  double* out;
  uint32_t nent, gsize, es, cs;
  uint32_t nch[4];
};

__device__ __forceinline__ void reduce_entry(const ReduceArgs& a, uint32_t e, uint32_t lane) {
  const uint32_t nc = a.nch[e / a.gsize];
  const double* p = a.in + (size_t)e * a.es;
  double v = 0.0;
  for (uint32_t c = lane; c < nc; c += 64) v += p[(size_t)c * a.cs];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) a.out[e] = v;
}

__global__ __launch_bounds__(256) void k_reduce_chunks(ReduceArgs a, Status s) {
  if (s.skip()) return;
  const uint32_t e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e < a.nent) reduce_entry(a, e, threadIdx.x & 63);
}

// Two independent sets of sums in one launch: the entries of b follow
// those of a.
__global__ __launch_bounds__(256) void k_reduce_chunks2(ReduceArgs a, ReduceArgs b, Status s) {
  if (s.skip()) return;
  const uint32_t e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e < a.nent) reduce_entry(a, e, threadIdx.x & 63);
  else if (e - a.nent < b.nent) reduce_entry(b, e - a.nent, threadIdx.x & 63);
}

// Column-side mode with a short side (I <= 128, K <= 64, R <= 8): instead
// of the K x K Gram, the leading left singular vectors of Y_(k) (I x K)
// come from a block subspace iteration on Y Y^T, with Y held in LDS in
// float64 and every product on float64 MFMA, in one workgroup:
//  - start: the previous solve's block of 16 orthonormal Ritz vectors,
//    passed once through the filter below on the previous theta_16; else
//    the current factor A_k (fixed coordinates, so the previous sweep's or
//    the HOSVD's factor is already close) completed by fixed pseudo-random
//    columns and made orthonormal by two Cholesky-QR passes (the first
//    shifted by 1e-15 tr/16);
//  - Rayleigh-Ritz on the block (16 x 16 Jacobi from the identity), stop
//    when the R leading residuals ||Y Y^T q - theta q|| are below 1e-10 of
//    theta_1;
//  - else twice a degree-2 Chebyshev filter on [0, theta_16] (two products
//    by Y Y^T, then two Cholesky-QR passes), and again.
// The Ritz vectors are the factor (sign rule as everywhere); theta are the
// squared singular values (the Gram's eigenvalues).
//
// The same iteration runs on a row-side Gram G = Y_(k) Y_(k)^T, one product
// by G in place of the two by Y, with the current factor as the cold start
// (fixed pseudo-random columns only, when there is none: the HOSVD):
//  - OP 1, side 33..64: G in LDS; it reports through `done` whether the
//    test passed, and if not, the caller's Jacobi solve of the same Gram
//    runs instead;
//  - OP 2, side 80..256 (a multiple of 16): G read from global memory (it
//    stays in L2 across the products), up to 16 Rayleigh-Ritz steps.
constexpr int kSsMaxI = 128, kSsMaxK = 64, kSsB = 16, kSsMaxIt = 8, kSsMaxIG = 256;

struct SsArgs {
  const float* Y;          // OP 0: view (O, I, Q) of Y_k: Y_(k)[i][o Q + q] = Y[(o I + i) Q + q]
  const double* G;         // OP 1, 2: the I x I Gram, row-major
  int32_t* done;           // OP 1: set to 1 when the residual test passed, else 0
  uint32_t O, I, Q, K, R;
  const double* Aprev;     // I x R, the current factor, or null
  double rtol, rfail;      // residual test (relative to theta_1): pass, and failure at the end
  double* state;           // I x 16: the block of the last solve
  double* lam;             // >= 16
  int32_t* tag;
  int32_t tagval;
  double* Aout;
  float* af;
  int32_t* stats;
  Status st;
};

// D (M x N) = op(A) B on float64 MFMA for LDS arrays with leading dims:
// op(A)[i][k] = TA ? A[k][i] : A[i][k]; M, N and Kd multiples of 16.  Each
// wave takes 16 x 16 output tiles, two at a time; the operands of four
// summation steps are read from LDS before their products.  D must not
// alias A or B.
template <int NT, bool TA>
__device__ void ss_mm(const double* A, int lda, const double* Bm, int ldb, double* D, int ldd, int M,
                      int N, int Kd) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int tn = N / 16, nt = (M / 16) * tn;
  for (int t0 = w; t0 < nt; t0 += 2 * NW) {
    const int t1 = t0 + NW;
    const bool two = t1 < nt;
    const int ti0 = t0 / tn, tj0 = t0 % tn, ti1 = (two ? t1 : t0) / tn, tj1 = (two ? t1 : t0) % tn;
    const int row0 = ti0 * 16 + li, row1 = ti1 * 16 + li, col0 = tj0 * 16 + li, col1 = tj1 * 16 + li;
    v4d c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Kd; k0 += 16) {
      double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + lk;
        a0[u] = TA ? A[k * lda + row0] : A[row0 * lda + k];
        a1[u] = TA ? A[k * lda + row1] : A[row1 * lda + k];
        b0[u] = Bm[k * ldb + col0];
        b1[u] = Bm[k * ldb + col1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], c1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      D[(ti0 * 16 + lk + 4 * v) * ldd + col0] = c0[v];
      if (two) D[(ti1 * 16 + lk + 4 * v) * ldd + col1] = c1[v];
    }
  }
  __syncthreads();
}

// D (M x 16, LDS) = A^T B for A in global memory (Kd x M, row-major, lda;
// the callers' A is symmetric, so this is A B) and B in LDS (Kd x 16); M and
// Kd multiples of 16.  A lane group reads 16 consecutive entries of a row
// of A, whole cache lines.  Each wave takes two 16-column tiles at a time
// and walks the summation index in chunks of 32 with two register sets: the
// A entries of the next chunk are requested from memory while the products
// of the current one run (B entries are read from LDS just before their
// products); a last half chunk of 16 is read directly.
template <int NT>
__device__ void ss_mm_ga(const double* __restrict__ A, int lda, const double* Bm, int ldb, double* D,
                         int ldd, int M, int Kd) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int nt = M / 16, nc = Kd / 32;
  const size_t step = (size_t)4 * lda;   // four summation indices
  for (int t0 = w; t0 < nt; t0 += 2 * NW) {
    const int t1 = t0 + NW;
    const bool two = t1 < nt;
    const double* r0 = A + (size_t)lk * lda + t0 * 16 + li;
    const double* r1 = A + (size_t)lk * lda + (two ? t1 : t0) * 16 + li;
    v4d c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    double x0[8], x1[8], y0[8], y1[8];
    auto load = [&](double* d0, double* d1, int k0) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        d0[u] = r0[(size_t)(k0 / 4 + u) * step];
        d1[u] = r1[(size_t)(k0 / 4 + u) * step];
      }
    };
    auto mul = [&](const double* s0, const double* s1, int k0) __attribute__((always_inline)) {
      double b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = Bm[(k0 + 4 * u + lk) * ldb + li];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(s0[u], b[u], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(s1[u], b[u], c1, 0, 0, 0);
      }
    };
    int c = 0;
    if (nc > 0) load(x0, x1, 0);
    for (; c + 1 < nc; c += 2) {
      load(y0, y1, (c + 1) * 32);
      mul(x0, x1, c * 32);
      load(x0, x1, (c + 2 < nc ? c + 2 : c + 1) * 32);
      mul(y0, y1, (c + 1) * 32);
    }
    if (c < nc) mul(x0, x1, c * 32);
    for (int k0 = nc * 32; k0 < Kd; k0 += 4) {   // the half chunk
      const double bv = Bm[(k0 + lk) * ldb + li];
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(r0[(size_t)(k0 / 4) * step], bv, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(r1[(size_t)(k0 / 4) * step], bv, c1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      D[(t0 * 16 + lk + 4 * v) * ldd + li] = c0[v];
      if (two) D[(t1 * 16 + lk + 4 * v) * ldd + li] = c1[v];
    }
  }
  __syncthreads();
}

template <int NT, int OP>
__global__ __launch_bounds__(NT) void k_mode_ss(SsArgs a) {
  constexpr bool GRAM = OP != 0;
  constexpr int MAXI = OP == 2 ? kSsMaxIG : kSsMaxI, MAXIT = OP == 2 ? 16 : kSsMaxIt;
  if (a.st.skip()) return;
  constexpr int B = kSsB, LB = B + 1, LK = kSsMaxK + 1;
  // Y (OP 0), G (OP 1); nothing for OP 2
  __shared__ double Y[OP == 0 ? kSsMaxI : (OP == 1 ? kSsMaxK : 1)][LK];
  __shared__ double Q0[MAXI][LB], Q1[MAXI][LB], Q2[MAXI][LB];
  __shared__ double W[OP == 0 ? kSsMaxK : 1][LB];
  __shared__ double S[B][LB];
  __shared__ double th[B], rinv[B], sgn[B];
  __shared__ double red[NT / 16][B];
  __shared__ int col_of_rank[B];
  __shared__ JacLds<16> J;
  const int tid = threadIdx.x;
  const int I = (int)a.I, K = (int)a.K, R = (int)a.R;
  const int Mp = (I + 15) / 16 * 16, Kp = (K + 15) / 16 * 16;
  // eight loads per thread issued before their LDS stores
  static_assert(kSsMaxI * kSsMaxK % (8 * NT) == 0, "Y load in groups of eight");
  if (OP == 1) {   // G (I x I, I <= 64) in Y, zero padded
    // unconditional loads at clamped indices (entries of G, finite), the
    // padding zeroed by a factor 0: a predicated load, or a select the
    // compiler turns back into one, is a branch that waits for the load
    constexpr int NL = kSsMaxK * kSsMaxK / NT;
    double g[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = u * NT + tid, i = e / kSsMaxK, k = e % kSsMaxK;
      g[u] = a.G[(size_t)min(i, I - 1) * I + min(k, I - 1)];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = u * NT + tid, i = e / kSsMaxK, k = e % kSsMaxK;
      Y[i][k] = g[u] * ((i < I && k < I) ? 1.0 : 0.0);
    }
  }
  for (int e0 = 0; e0 < (GRAM ? 0 : kSsMaxI * kSsMaxK); e0 += 8 * NT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT + tid, i = e / kSsMaxK, k = e % kSsMaxK;
      v[u] = 0.0f;
      if (i < I && k < K) {
        const uint32_t o = (uint32_t)k / a.Q, q = (uint32_t)k % a.Q;
        v[u] = a.Y[((size_t)o * a.I + i) * a.Q + q];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT + tid;
      Y[e / kSsMaxK][e % kSsMaxK] = (double)v[u];
    }
  }
  // Start block: the previous solve's block (warm), else the current factor
  // completed by fixed pseudo-random columns, else those columns only.  The
  // source is the same for every thread; within it the eight loads of a
  // thread are unconditional, at indices clamped into the source (finite
  // values), and rows past I are zeroed by a factor 0.
  const bool warm = *a.tag == a.tagval;
  const int src = warm ? 0 : (a.Aprev ? 1 : 2);
  auto hashval = [](int i, int j) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(j + 1) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (double)(h >> 8) * (1.0 / 16777216.0) - 0.5;
  };
  static_assert(MAXI * B % (8 * NT) == 0, "start block loaded eight values per thread at a time");
  for (int e0 = 0; e0 < MAXI * B; e0 += 8 * NT) {
    double v[8];
    if (src == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * NT + tid, i = e / B, j = e % B;
        v[u] = a.state[min(i, I - 1) * B + j];
      }
    } else if (src == 1) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * NT + tid, i = e / B, j = e % B;
        v[u] = a.Aprev[(size_t)min(i, I - 1) * R + min(j, R - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT + tid, i = e / B, j = e % B;
      const double row = i < I ? 1.0 : 0.0;
      double x;
      if (src == 0) {
        x = v[u] * row;
      } else if (src == 1) {
        const double own = j < R ? 1.0 : 0.0;
        x = (v[u] * own + hashval(i, j) * (1.0 - own)) * row;
      } else {
        x = hashval(i, j) * row;
      }
      Q0[e / B][e % B] = x;
    }
  }
  __syncthreads();
  double (*Qc)[LB] = Q0, (*Za)[LB] = Q1, (*Zb)[LB] = Q2;
  // two Cholesky-QR passes on the block P (Mp x 16), in place
  auto orth = [&](double (*P)[LB]) __attribute__((always_inline)) {
    for (int pass = 0; pass < 2; ++pass) {
      ss_mm<NT, true>(&P[0][0], LB, &P[0][0], LB, &S[0][0], LB, B, B, Mp);
      if (tid < 64) {
        double tr = tid < B ? S[tid][tid] : 0.0;
        for (int o = 8; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
        double av[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) av[k] = tid < 16 ? S[tid][k] : 0.0;
        if (pass == 0)
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (k == tid) av[k] += 1e-15 * tr / B;
        chol16_wave(av, tid);
        if (tid < 16) {
          double dgl = 1.0;
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            S[tid][k] = av[k];
            if (k == tid) dgl = av[k];
          }
          rinv[tid] = 1.0 / dgl;
        }
      }
      __syncthreads();
      for (int i = tid; i < Mp; i += NT) {
        double q[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          double v = P[i][j];
#pragma unroll
          for (int k = 0; k < j; ++k) v = fma(-q[k], S[j][k], v);
          q[j] = v * rinv[j];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) P[i][j] = q[j];
      }
      __syncthreads();
    }
  };
  // D = Y (Y^T P), or D = G P
  auto gq = [&](double (*P)[LB], double (*D)[LB]) __attribute__((always_inline)) {
    if (OP == 2) {
      ss_mm_ga<NT>(a.G, I, &P[0][0], LB, &D[0][0], LB, Mp, Mp);
    } else if (OP == 1) {
      ss_mm<NT, false>(&Y[0][0], LK, &P[0][0], LB, &D[0][0], LB, Mp, B, Mp);
    } else {
      ss_mm<NT, true>(&Y[0][0], LK, &P[0][0], LB, &W[0][0], LB, Kp, B, Mp);
      ss_mm<NT, false>(&Y[0][0], LK, &W[0][0], LB, &D[0][0], LB, Mp, B, Kp);
    }
  };
  // degree-2 Chebyshev filter on [0, tau] applied to the block Qc, then two
  // Cholesky-QR passes (plain steps if tau is not a usable bound)
  auto filter = [&](double tau, double ref) __attribute__((always_inline)) {
    const bool cheb = tau > 1e-12 * ref && isfinite(tau);
    const double a1 = cheb ? 2.0 / tau : 1.0, b1 = cheb ? -1.0 : 0.0;
    const double a2 = cheb ? 4.0 / tau : 1.0, b2 = cheb ? -2.0 : 0.0, c2 = cheb ? -1.0 : 0.0;
    gq(Qc, Za);
    for (int e = tid; e < Mp * B; e += NT) {
      const int i = e / B, j = e % B;
      Za[i][j] = a1 * Za[i][j] + b1 * Qc[i][j];
    }
    __syncthreads();
    gq(Za, Zb);
    for (int e = tid; e < Mp * B; e += NT) {
      const int i = e / B, j = e % B;
      Zb[i][j] = a2 * Zb[i][j] + b2 * Za[i][j] + c2 * Qc[i][j];
    }
    __syncthreads();
    {
      double (*t)[LB] = Qc;
      Qc = Zb;
      Zb = t;
    }
    orth(Qc);
  };
  // Warm: the previous block holds orthonormal Ritz vectors of the previous
  // matrix, so two applications of the filter (on the previous theta_16)
  // go first and the first Rayleigh-Ritz step already sees the filtered
  // block (after one, the test failed in every steady-state sweep; a
  // Rayleigh-Ritz step between the two would not change their span).
  if (!warm) orth(Qc);
  if (warm) {
    const double tau0 = a.lam[B - 1], ref0 = a.lam[0];
    if (tau0 > 1e-12 * ref0 && isfinite(tau0)) {
      filter(tau0, ref0);
      // one application is enough for the looser test of mixed-precision inputs
      if (a.rtol < 1e-7) filter(tau0, ref0);
    }
  }
  bool conv = false;
  int it = 0;
  double worst = 0.0, ref = 0.0;
  for (;; ++it) {
    // Rayleigh-Ritz: Z = G Q, H = Q^T Z, H = V Theta V^T
    gq(Qc, Za);
    ss_mm<NT, true>(&Qc[0][0], LB, &Za[0][0], LB, &J.A[0][0], 17, B, B, Mp);
    for (int e = tid; e < 16 * 16; e += NT) {
      const int x = e / 16, y = e % 16;
      if (x < y) {
        const double m = 0.5 * (J.A[x][y] + J.A[y][x]);
        J.A[x][y] = m;
        J.A[y][x] = m;
      }
    }
    __syncthreads();
    jacobi_setup<16, NT>(J, 16, false, nullptr);
    bool jc;
    jacobi_core<16, NT>(J, 16, R, &jc, 1e-24);
    jacobi_sort_store<16, NT>(J, 16, nullptr, nullptr);
    if (tid < 16) col_of_rank[J.rk[tid]] = tid;
    __syncthreads();
    if (tid < 16) th[tid] = J.A[col_of_rank[tid]][col_of_rank[tid]];
    for (int e = tid; e < 16 * 16; e += NT) {   // sorted eigenvectors into J.W
      const int x = e / 16, r = e % 16;
      J.W[x][r] = J.V[x][col_of_rank[r]];
    }
    __syncthreads();
    ss_mm<NT, false>(&Qc[0][0], LB, &J.W[0][0], 17, &Zb[0][0], LB, Mp, B, B);   // Ritz vectors
    ss_mm<NT, false>(&Za[0][0], LB, &J.W[0][0], 17, &Qc[0][0], LB, Mp, B, B);   // G times them
    {
      // residuals of the R leading pairs: column r = tid % 16, rows by part
      const int r = tid % 16, part = tid / 16;
      double acc = 0.0;
      if (r < R)
        for (int i = part; i < Mp; i += NT / 16) {
          const double d = Qc[i][r] - th[r] * Zb[i][r];
          acc = fma(d, d, acc);
        }
      red[part][r] = acc;
    }
    __syncthreads();
    worst = 0.0;
    for (int r = 0; r < R; ++r) {
      double s2 = 0.0;
      for (int p = 0; p < NT / 16; ++p) s2 += red[p][r];
      worst = fmax(worst, sqrt(s2));
    }
    ref = fabs(th[0]);
    {
      double (*t)[LB] = Qc;   // the Ritz vectors become the block
      Qc = Zb;
      Zb = t;
    }
    conv = worst <= a.rtol * ref;
    if (conv || it == MAXIT - 1) break;
    // tau = theta_16; two applications between Rayleigh-Ritz steps (one
    // seldom sufficed, and the step between would not change the span)
    filter(th[B - 1], ref);
    filter(th[B - 1], ref);
  }
  // OP 1: a block that did not pass the test is dropped (the Jacobi solve
  // of the caller runs instead and leaves its own warm-start tag)
  if (OP == 1) {
    const bool ok = conv || worst <= a.rfail * ref;
    if (tid == 0) *a.done = ok ? 1 : 0;
    if (!ok) return;
  }
  // sign rule and stores; the block is kept for the next solve
  if (tid < R) {
    double best = -1.0, val = 0.0;
    for (int i = 0; i < I; ++i) {
      const double v = Qc[i][tid];
      if (fabs(v) > best) {
        best = fabs(v);
        val = v;
      }
    }
    sgn[tid] = val < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < I * 16; e += NT) {
    const int i = e / 16, r = e % 16;
    const double v = r < R ? sgn[r] * Qc[i][r] : 0.0;
    if (r < R) a.Aout[(size_t)i * R + r] = v;
    a.af[e] = (float)v;
    a.state[i * B + r] = Qc[i][r];
  }
  if (tid < B) a.lam[tid] = th[tid];
  if (tid == 0) {
    *a.tag = a.tagval;
    if (a.stats) *a.stats = 3000 + it + 1;
    if (OP != 1 && !conv && worst > a.rfail * ref) atomicCAS(a.st.st, 0, MACH_ENOCONV);
    if (OP == 0 && !(th[R - 1] > 1e-13 * th[0])) atomicCAS(a.st.st, 0, MACH_EDEGENERATE);
  }
}

// One mode update of a HOOI sweep, sides up to 64, in one workgroup:
// G = sum of the Gram partials (fixed order); warm-started Jacobi; the
// eigenpairs sorted and kept for the next sweep.  Row-side Gram: the top R
// eigenvectors are the factor; the sign rule is applied and the float64
// factor and its float32 copy stored.  Column-side Gram: M = V_R
// Lambda_R^{-1/2} (s x 16) is written for the back-projection kernels.
struct SolveArgs {
  const double* part;
  uint32_t nchunk, s, I, R;
  int kside;
  const double* ctc;      // column side: C_j partials of the other modes (k_ctc_partial), or null
  uint32_t cstride;       // entry stride of ctc (chunks per entry)
  int nother;              // other modes: ranks, column strides in Y_(k), C_j chunks
  uint32_t oR[3], ost[3], onch[3];
  double* V;
  double* lam;
  int32_t* tag;
  int32_t tagval;
  double* M;
  double* Aout;
  float* af;
  int32_t* stats;
  double tol2;            // Jacobi stopping threshold (off-diagonal / diagonal mass)
  Status st;
};

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_mode_solve(SolveArgs a) {
  if (a.st.skip()) return;
  __shared__ JacLds<NP> L;
  __shared__ double sgn[16];
  __shared__ int col_of_rank[16];
  const int n = (int)a.s, tid = threadIdx.x;
  load_gram<NP, NT>(L.A, n, a.part, a.nchunk);
  __syncthreads();
  bool warm = (*a.tag == a.tagval);
  if (warm && a.ctc) {
    __shared__ double Cj[3][16][17];
    for (int e = tid; e < a.nother * 256; e += NT) {
      const double* p = a.ctc + (size_t)e * a.cstride;
      const uint32_t nc = a.onch[e >> 8];
      double v = 0.0;
#pragma unroll 8
      for (uint32_t c = 0; c < nc; ++c) v += p[c];
      Cj[e >> 8][(e >> 4) & 15][e & 15] = v;
    }
    load_basis<NP, NT>(L.V, n, true, a.V);
    __syncthreads();
    // P[x][y] = prod_j C_j[(x / st_j) % R_j][(y / st_j) % R_j]
    for (int e = tid; e < NP * NP; e += NT) {
      const int x = e / NP, y = e % NP;
      double v = (x == y) ? 1.0 : 0.0;
      if (x < n && y < n) {
        v = 1.0;
        for (int j = 0; j < a.nother; ++j)
          v *= Cj[j][(x / a.ost[j]) % a.oR[j]][(y / a.ost[j]) % a.oR[j]];
      }
      L.W[x][y] = v;
    }
    __syncthreads();
    // V <- P^T V_old
    lds_gemm<NP, NT, true>(L.W, L.V, L.V);
    // Newton-Schulz steps towards the nearest orthogonal matrix,
    // V <- V (3 I - V^T V) / 2, until ||V^T V - I||_F <= 1e-11 (at most 10;
    // if the factors moved so far that it does not get there, cold start).
    bool ortho = false;
    for (int it = 0; it < 11; ++it) {
      lds_gemm<NP, NT, true>(L.V, L.V, L.W);
      double dev2 = 0.0, unused = 0.0;
      for (int e = tid; e < NP * NP; e += NT) {
        const int x = e / NP, y = e % NP;
        const double d = L.W[x][y] - (x == y ? 1.0 : 0.0);
        dev2 = fma(d, d, dev2);
        L.W[x][y] = 0.5 * ((x == y ? 3.0 : 0.0) - L.W[x][y]);
      }
      block_sum2n<NT>(dev2, unused, L.red);
      if (dev2 <= 1e-22) {
        ortho = true;
        break;
      }
      if (it == 10) break;
      lds_gemm<NP, NT, false>(L.V, L.W, L.V);
    }
    if (!ortho) {
      for (int e = tid; e < NP * NP; e += NT) L.V[e / NP][e % NP] = (e / NP == e % NP) ? 1.0 : 0.0;
      __syncthreads();
    }
    warm = ortho;
    jacobi_setup<NP, NT>(L, n, ortho, nullptr, true);
  } else {
    jacobi_setup<NP, NT>(L, n, warm, a.V);
  }
  bool conv;
  int used = jacobi_core<NP, NT>(L, n, (int)a.R, &conv, a.tol2);
  jacobi_sort_store<NP, NT>(L, n, a.lam, a.V);
  if (tid == 0 && a.stats) *a.stats = used + (warm && a.ctc ? 2000 : warm ? 1000 : 0);
  if (tid < n && L.rk[tid] < (int)a.R) col_of_rank[L.rk[tid]] = tid;
  __syncthreads();
  if (tid == 0) {
    *a.tag = a.tagval;
    if (!conv) atomicCAS(a.st.st, 0, MACH_ENOCONV);
  }
  if (a.kside) {
    if (tid == 0) {
      double l0 = L.A[col_of_rank[0]][col_of_rank[0]];
      double lr = L.A[col_of_rank[a.R - 1]][col_of_rank[a.R - 1]];
      if (!(lr > 1e-13 * l0)) atomicCAS(a.st.st, 0, MACH_EDEGENERATE);
    }
    for (int e = tid; e < n * 16; e += NT) {
      int x = e >> 4, r = e & 15;
      double v = 0.0;
      if (r < (int)a.R) {
        int col = col_of_rank[r];
        v = L.V[x][col] / sqrt(fmax(L.A[col][col], 1e-300));
      }
      a.M[e] = v;
    }
    return;
  }
  // row side: factor = top R eigenvectors (I == n rows); sign rule per column
  if (tid < (int)a.R) {
    int col = col_of_rank[tid];
    double best = -1.0, val = 0.0;
    for (int x = 0; x < n; ++x) {
      double v = L.V[x][col];
      if (fabs(v) > best) {
        best = fabs(v);
        val = v;
      }
    }
    sgn[tid] = val < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < n * 16; e += NT) {
    int x = e >> 4, r = e & 15;
    double v = r < (int)a.R ? sgn[r] * L.V[x][col_of_rank[r]] : 0.0;
    if (r < (int)a.R) a.Aout[(size_t)x * a.R + r] = v;
    a.af[e] = (float)v;
  }
}

// Column-side back-projection Aw = Y_(k) M (I x 16, float64) from the
// float32 view (O, I, Q) of Y_k, plus per-workgroup partials of Aw^T Aw.
// Workgroups from nwg on copy the other modes' float32 factors for the next
// sweep's warm start instead (snapshot; they take no part in the rest).
__global__ __launch_bounds__(256) void k_bp_tall(const float* __restrict__ Y, uint32_t O, uint32_t I,
                                                 uint32_t Q, const double* __restrict__ M, uint32_t R,
                                                 double* __restrict__ Aw, double* __restrict__ part,
                                                 uint32_t nwg, SnapArgs sa, uint32_t snap_wg,
                                                 Status s) {
  if (s.skip()) return;
  if (blockIdx.x >= nwg) {   // whole workgroups, before any barrier
    const uint32_t b = blockIdx.x - nwg, j = b / snap_wg;
    const uint32_t e = (b % snap_wg) * 256 + threadIdx.x;
    if ((int)j < sa.n && e < sa.n4[j]) sa.dst[j][e] = sa.src[j][e];
    return;
  }
  __shared__ double Ms[256][17];
  __shared__ double rows[256][17];
  const uint32_t K = O * Q;
  {
    // M (K x 16, K <= 256) staged with unconditional loads at clamped
    // indices; the rows from K on (unused) get zeros
    double mv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) mv[t] = M[min(threadIdx.x + 256u * t, K * 16 - 1)];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const uint32_t e = threadIdx.x + 256u * t;
      Ms[e >> 4][e & 15] = mv[t] * (e < K * 16 ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  double acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;
  if (i < I) {
    for (uint32_t o = 0; o < O; ++o) {
      const float* yrow = Y + ((size_t)o * I + i) * Q;
      // eight entries of the row per round, loaded before any is used
      // (clamped to the row; the extra ones weigh 0)
      for (uint32_t q0 = 0; q0 < Q; q0 += 8) {
        float yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = yrow[min(q0 + u, Q - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double y = (double)yv[u] * (q0 + u < Q ? 1.0 : 0.0);
          const uint32_t kappa = o * Q + min(q0 + u, Q - 1);
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[r] = fma(y, Ms[kappa][r], acc[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) Aw[(size_t)i * 16 + r] = (uint32_t)r < R ? acc[r] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) rows[threadIdx.x][r] = (i < I && (uint32_t)r < R) ? acc[r] : 0.0;
  __syncthreads();
  const int x = threadIdx.x >> 4, y = threadIdx.x & 15;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
  for (int t = 0; t < 256; t += 4) {
    g0 = fma(rows[t][x], rows[t][y], g0);
    g1 = fma(rows[t + 1][x], rows[t + 1][y], g1);
    g2 = fma(rows[t + 2][x], rows[t + 2][y], g2);
    g3 = fma(rows[t + 3][x], rows[t + 3][y], g3);
  }
  part[(size_t)blockIdx.x * 256 + threadIdx.x] = (g0 + g1) + (g2 + g3);
}

// One Cholesky-QR pass on Aw (I x 16): every workgroup sums the Gram
// partials (fixed order), factors S = L L^T in one wave (registers), and
// replaces each of its rows a by the solution q of q L^T = a; then writes
// per-workgroup column maxima of |q| for the sign rule.
__global__ __launch_bounds__(256) void k_chol_apply_tall(double* __restrict__ Aw, uint32_t I, uint32_t R,
                                                         const double* __restrict__ part, uint32_t nchunk,
                                                         double* __restrict__ pv, uint32_t* __restrict__ pi,
                                                         Status s) {
  if (s.skip()) return;
  __shared__ double S[16][17];
  __shared__ double rinv[16];
  __shared__ double bv[256];
  __shared__ uint32_t bi[256];
  const int tid = threadIdx.x;
  {
    double g = 0.0;
    for (uint32_t c = 0; c < nchunk; ++c) g += part[(size_t)c * 256 + tid];
    const int x = tid >> 4, y = tid & 15;
    // columns at or beyond R are zero: factor the identity there
    S[x][y] = (x < (int)R && y < (int)R) ? g : (x == y ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < 64) {
    const int x = tid;
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = x < 16 ? S[x][k] : 0.0;
    chol16_wave(a, x);
    if (x < 16) {
      double dgl = 1.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        S[x][k] = a[k];
        if (k == x) dgl = a[k];
      }
      rinv[x] = 1.0 / dgl;
    }
  }
  __syncthreads();
  const uint32_t i = blockIdx.x * 256 + tid;
  double out[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) out[r] = 0.0;
  if (i < I) {
    double a[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = Aw[(size_t)i * 16 + r];
    // forward substitution: out_j = (a_j - sum_{k < j} out_k L[j][k]) / L[j][j]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double v = a[j];
#pragma unroll
      for (int k = 0; k < j; ++k) v = fma(-out[k], S[j][k], v);
      out[j] = (uint32_t)j < R ? v * rinv[j] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) Aw[(size_t)i * 16 + r] = out[r];
  }
  // column maxima over this workgroup's rows (value, then lowest row):
  // |q| through LDS, thread (g, c) scans rows g, g + 16, ... of column c in
  // increasing order, then 16 threads take the 16 group results in order.
  __shared__ double aq[256][17];
#pragma unroll
  for (int r = 0; r < 16; ++r) aq[tid][r] = i < I ? fabs(out[r]) : -1.0;
  __syncthreads();
  {
    const int cidx = tid & 15, g = tid >> 4;
    double v = -1.0;
    uint32_t ix = 0xffffffffu;
    for (int row = g; row < 256; row += 16) {
      const double x = aq[row][cidx];
      if (x > v) {
        v = x;
        ix = blockIdx.x * 256 + row;
      }
    }
    bv[tid] = v;
    bi[tid] = ix;
  }
  __syncthreads();
  if (tid < 16) {
    double v = -1.0;
    uint32_t ix = 0xffffffffu;
    for (int g = 0; g < 16; ++g) {
      const double v2 = bv[g * 16 + tid];
      const uint32_t i2 = bi[g * 16 + tid];
      if (v2 > v || (v2 == v && i2 < ix)) {
        v = v2;
        ix = i2;
      }
    }
    pv[blockIdx.x * 16 + tid] = v;
    pi[blockIdx.x * 16 + tid] = ix;
  }
}

// ---------------------------------------------------------------------------
// Dense float64 helpers for the subspace solver and CholeskyQR2
// ---------------------------------------------------------------------------

// C[M x N] = A[M x K] * B[K x N] (row-major, leading dims), N <= 64.  A
// workgroup owns 16 rows; thread (row, column group of 4).
__global__ __launch_bounds__(256) void k_gemm64(const double* __restrict__ A, uint32_t lda,
                                                const double* __restrict__ B, uint32_t ldb,
                                                double* __restrict__ C, uint32_t ldc, uint32_t M,
                                                uint32_t K, uint32_t N, Status s) {
  if (s.skip()) return;
  __shared__ double As[16][65];
  __shared__ double Bs[64][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const uint32_t m0 = blockIdx.x * 16;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t k0 = 0; k0 < K; k0 += 64) {
    // all tile loads issued before any is stored: unconditional, at indices
    // clamped into A and B (finite), the outside entries zeroed by a factor 0
    double va[4], vb[16];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = threadIdx.x + 256 * t, r = e >> 6, c = e & 63;
      va[t] = A[(size_t)min(m0 + r, M - 1) * lda + min(k0 + c, K - 1)];
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = threadIdx.x + 256 * t, r = e >> 6, c = e & 63;
      vb[t] = B[(size_t)min(k0 + r, K - 1) * ldb + min((uint32_t)c, N - 1)];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = threadIdx.x + 256 * t, r = e >> 6, c = e & 63;
      As[r][c] = va[t] * ((m0 + r < M && k0 + c < K) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = threadIdx.x + 256 * t, r = e >> 6, c = e & 63;
      Bs[r][c] = vb[t] * ((k0 + r < K && (uint32_t)c < N) ? 1.0 : 0.0);
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 64; ++kk) {
      double u = As[ty][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = fma(u, Bs[kk][tx * 4 + j], acc[j]);
    }
    __syncthreads();
  }
  uint32_t m = m0 + ty;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t n = tx * 4 + j;
    if (m < M && n < N) C[(size_t)m * ldc + n] = acc[j];
  }
}

// part[x][y][chunk] = sum over the chunk's rows m of A[m][x] * B[m][y]  (x, y < n <= 64;
// chunk-minor, so that a consumer reads the partials of one entry contiguously)
__global__ __launch_bounds__(256) void k_atb_partial(const double* __restrict__ A, uint32_t lda,
                                                     const double* __restrict__ B, uint32_t ldb,
                                                     uint32_t M, uint32_t n, uint32_t rows,
                                                     double* __restrict__ part, Status s) {
  if (s.skip()) return;
  __shared__ double As[32][65];
  __shared__ double Bs[32][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const uint32_t r0 = blockIdx.x * rows, r1 = min(M, r0 + rows);
  double acc[4][4] = {};
  for (uint32_t m0 = r0; m0 < r1; m0 += 32) {
    // loads unconditional at clamped indices (finite), then stored with the
    // outside entries zeroed by a factor 0
    double va[8], vb[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = threadIdx.x + 256 * t, r = e >> 6, c = e & 63;
      const size_t mm = min(m0 + r, r1 - 1), cc = min((uint32_t)c, n - 1);
      va[t] = A[mm * lda + cc];
      vb[t] = B[mm * ldb + cc];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = threadIdx.x + 256 * t, r = e >> 6, c = e & 63;
      const double ok = (m0 + r < r1 && (uint32_t)c < n) ? 1.0 : 0.0;
      As[r][c] = va[t] * ok;
      Bs[r][c] = vb[t] * ok;
    }
    __syncthreads();
    for (int rr = 0; rr < 32; ++rr) {
      double u[4], w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        u[i] = As[rr][tx * 4 + i];
        w[i] = Bs[rr][ty * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(u[i], w[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t x = tx * 4 + i, y = ty * 4 + j;
      if (x < n && y < n) part[(size_t)(x * n + y) * gridDim.x + blockIdx.x] = acc[i][j];
    }
}

// Degree-2 Chebyshev filter of the subspace iteration, applied as the
// epilogue of the products by G: with tau the smallest Ritz value of the last
// Rayleigh-Ritz step, t(x) = 2 x / tau - 1 maps [0, tau] onto [-1, 1], and
// two steps give T_2(t(G)) X = 2 t(G) Y1 - X with Y1 = t(G) X, which damps
// every eigenvalue below tau to at most 1 while the wanted ones grow like
// 8 (lambda / tau)^2 (plain power steps grow them like (lambda / tau)^2).
// out = alpha G X + beta X + gamma Xp: step 1 (2 / tau, -1, 0), step 2
// (4 / tau, -2, -1) with X = Y1 and Xp the first step's input; plain
// (1, 0, 0) until a Ritz value is known (*valid == 0) or if tau <= 0.
struct Cheb {
  int step;               // 0: plain product, 1 or 2: filter step
  const double* lam;      // Ritz values of the last Rayleigh-Ritz step
  uint32_t bidx;          // index of the smallest one (block size - 1)
  const int32_t* valid;   // nonzero once lam holds Ritz values
  const double* Xp;       // input of step 1 (step 2 only), ld kBlock
};

struct ChebCoef {
  double al, be, ga;
};

__device__ __forceinline__ ChebCoef cheb_coef(const Cheb& ch) {
  if (ch.step == 0 || !ch.valid || *ch.valid == 0) return ChebCoef{1.0, 0.0, 0.0};
  const double tau = ch.lam[ch.bidx];
  if (!(tau > 0.0) || !isfinite(tau)) return ChebCoef{1.0, 0.0, 0.0};
  if (ch.step == 1) return ChebCoef{2.0 / tau, -1.0, 0.0};
  return ChebCoef{4.0 / tau, -2.0, -1.0};
}

// C[M x N] partials of A[M x K] * B[K x N] (row-major, N <= NC) for long K:
// workgroup (x, y) owns rows 64x..64x+63 and the summation slice
// [y * kSplitK, (y + 1) * kSplitK) (a single slice covers all of K);
// P[y][m][0..63] (columns >= N are 0).  Tiles of 32 summation indices are
// staged in LDS (A transposed); each thread accumulates a block of
// 64 / (256 / (NC / 4)) rows x 4 columns in float64 (4 x 4 for NC = 64,
// 2 x 4 for NC = 32).
// One 32-index tile of the split product: A rows m0..m0+63, B columns
// 0..NC-1.  Loads are unconditional, at indices clamped into A and B (a
// predicated load, or a select that the compiler turns back into one, is
// compiled to a branch that waits for the load); splitk_stage zeroes the
// entries outside the tile by a factor 0 when it stores them to LDS, so
// that nothing waits for the loads before then.
template <int NC>
__device__ __forceinline__ void splitk_fetch(const double* __restrict__ A, uint32_t lda,
                                             const double* __restrict__ B, uint32_t ldb, uint32_t M,
                                             uint32_t N, uint32_t m0, uint32_t kc, uint32_t k1, int tid,
                                             double (&va)[8], double (&vb)[NC / 8]) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int e = tid + 256 * t, r = e >> 5, kk = e & 31;
    va[t] = A[(size_t)min(m0 + r, M - 1) * lda + min(kc + kk, k1 - 1)];
  }
#pragma unroll
  for (int t = 0; t < NC / 8; ++t) {
    const int e = tid + 256 * t, kb = e / NC, cb = e % NC;
    vb[t] = B[(size_t)min(kc + kb, k1 - 1) * ldb + min((uint32_t)cb, N - 1)];
  }
}

template <int NC>
__device__ __forceinline__ void splitk_stage(double (*As)[68], double (*Bs)[68], uint32_t M, uint32_t N,
                                             uint32_t m0, uint32_t kc, uint32_t k1, int tid,
                                             const double (&va)[8], const double (&vb)[NC / 8]) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int e = tid + 256 * t, r = e >> 5, kk = e & 31;
    As[kk][r] = va[t] * ((m0 + r < M && kc + kk < k1) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int t = 0; t < NC / 8; ++t) {
    const int e = tid + 256 * t, kb = e / NC, cb = e % NC;
    Bs[kb][cb] = vb[t] * ((kc + kb < k1 && (uint32_t)cb < N) ? 1.0 : 0.0);
  }
}

template <int NC>
__global__ __launch_bounds__(256) void k_gemm_splitk(const double* __restrict__ A, uint32_t lda,
                                                     const double* __restrict__ B, uint32_t ldb,
                                                     double* __restrict__ P, uint32_t M, uint32_t K,
                                                     uint32_t N, Cheb ch, Status s) {
  constexpr int TXN = NC / 4, TYN = 256 / TXN, TR = 64 / TYN;
  static_assert(TXN * TYN == 256 && TR * TYN == 64, "tile shape");
  if (s.skip()) return;
  __shared__ double As[32][68];
  __shared__ double Bs[32][68];
  const int tid = threadIdx.x, tx = tid % TXN, ty = tid / TXN;
  const uint32_t m0 = blockIdx.x * 64, k0 = blockIdx.y * kSplitK;
  const uint32_t k1 = gridDim.y == 1 ? K : min(K, k0 + kSplitK);
  double acc[TR][4];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // the next tile's loads are in flight while the current one is multiplied
  double va[8], vb[NC / 8];
  if (k0 < k1) splitk_fetch<NC>(A, lda, B, ldb, M, N, m0, k0, k1, tid, va, vb);
  for (uint32_t kc = k0; kc < k1; kc += 32) {
    splitk_stage<NC>(As, Bs, M, N, m0, kc, k1, tid, va, vb);
    __syncthreads();
    if (kc + 32 < k1) splitk_fetch<NC>(A, lda, B, ldb, M, N, m0, kc + 32, k1, tid, va, vb);
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      double a[TR], b[4];
#pragma unroll
      for (int i = 0; i < TR; ++i) a[i] = As[kk][ty * TR + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* o = P + ((size_t)blockIdx.y * M + m0) * 64;
  // single slice: P is the output, with the filter epilogue
  const ChebCoef cf = gridDim.y == 1 ? cheb_coef(ch) : ChebCoef{1.0, 0.0, 0.0};
  const double al = cf.al, be = cf.be, ga = cf.ga;
  if (NC < 64)   // the columns this variant does not compute
    for (int e = tid; e < 64 * (64 - NC); e += 256) {
      const uint32_t r = e / (64 - NC), cidx = NC + e % (64 - NC);
      if (m0 + r < M) o[(size_t)r * 64 + cidx] = 0.0;
    }
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const uint32_t r = ty * TR + i;
    if (m0 + r < M)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const size_t e = (size_t)(m0 + r) * ldb + tx * 4 + j;
        double v = al * acc[i][j];
        if (be != 0.0) v = fma(be, B[e], v);
        if (ga != 0.0) v = fma(ga, ch.Xp[e], v);
        o[(size_t)r * 64 + tx * 4 + j] = v;
      }
  }
}

// C[m][n] = sum over the nks slices of P[slice][m][n] (fixed order), n < 64,
// then the filter epilogue (X: the product's right operand, ld ldc).
__global__ void k_splitk_reduce(const double* __restrict__ P, uint32_t nks, uint32_t M,
                                double* __restrict__ C, uint32_t ldc, const double* __restrict__ X,
                                Cheb ch, Status s) {
  if (s.skip()) return;
  const uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= M * 64) return;
  // the slices in order, eight loads in flight (unconditional, clamped to
  // the last slice; a slice past the end adds +-0, which changes no sum)
  double acc = 0.0;
  for (uint32_t k0 = 0; k0 < nks; k0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(size_t)min(k0 + u, nks - 1) * M * 64 + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u] * (k0 + u < nks ? 1.0 : 0.0);
  }
  const ChebCoef cf = cheb_coef(ch);
  const double al = cf.al, be = cf.be, ga = cf.ga;
  const size_t o = (size_t)(e >> 6) * ldc + (e & 63);
  double v = al * acc;
  if (be != 0.0) v = fma(be, X[o], v);
  if (ga != 0.0) v = fma(ga, ch.Xp[o], v);
  C[o] = v;
}

// Cholesky-QR helper for an n x n Gram (n <= 64) summed from its chunk-minor
// partials, with shift * trace / n added to the diagonal: S = L L^T and
// B = L^{-T} (row-major n x n), both by 16 x 16 blocks.  A diagonal block is
// factored by one wave in registers; panel solves and trailing updates use
// all 256 threads; the inverse takes the diagonal blocks first (one wave
// each) and then one block row at a time.  Indices at or beyond n are padded
// with the identity.
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ part, uint32_t nchunk,
                                                  uint32_t n, double shift, double* __restrict__ B,
                                                  Status s) {
  if (s.skip()) return;
  __shared__ double A[64][65];    // S, factored in place into L (upper part zero)
  __shared__ double Li[64][65];   // L^{-1}
  __shared__ double T[64][65];    // block-row products
  __shared__ double trs;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nn = (int)n, nb = (nn + 15) / 16, E = nb * 16;
  {
    // S summed from its partials in chunk order, the 16 entries of a thread
    // loaded together (unconditionally, at indices clamped into the n x n
    // partials, the outside ones zeroed by a factor 0), then the padding
    // set to the identity
    constexpr int NE = 64 * 64 / 256;
    double g[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) g[u] = 0.0;
    for (uint32_t ch = 0; ch < nchunk; ++ch) {
      double pv[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = tid + 256 * u, r = e >> 6, c = e & 63;
        pv[u] = part[(size_t)(min(r, nn - 1) * nn + min(c, nn - 1)) * nchunk + ch];
      }
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = tid + 256 * u, r = e >> 6, c = e & 63;
        g[u] += pv[u] * ((r < nn && c < nn) ? 1.0 : 0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e >> 6, c = e & 63;
      A[r][c] = (r < nn && c < nn) ? g[u] : (r == c ? 1.0 : 0.0);
      Li[r][c] = 0.0;
    }
  }
  __syncthreads();
  if (tid < 64) {
    double tr = lane < nn ? A[lane][lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
    if (lane == 0) trs = tr;
  }
  __syncthreads();
  if (tid < nn) A[tid][tid] += shift * trs / n;
  __syncthreads();
  for (int K = 0; K < nb; ++K) {
    const int k0 = K * 16, m = E - k0 - 16;
    if (w == 0) {
      double a[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) a[k] = lane < 16 ? A[k0 + lane][k0 + k] : 0.0;
      chol16_wave(a, lane);
      if (lane < 16)
#pragma unroll
        for (int k = 0; k < 16; ++k) A[k0 + lane][k0 + k] = a[k];
    }
    __syncthreads();
    if (tid < m) {   // panel row r: solve l L_KK^T = A[r][k0 : k0 + 16]
      const int r = k0 + 16 + tid;
      double q[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double v = A[r][k0 + j];
#pragma unroll
        for (int k = 0; k < j; ++k) v = fma(-q[k], A[k0 + j][k0 + k], v);
        q[j] = v / A[k0 + j][k0 + j];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        A[r][k0 + j] = q[j];
        A[k0 + j][r] = 0.0;
      }
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += 256) {   // trailing lower part -= panel panel^T
      const int x = k0 + 16 + e / m, y = k0 + 16 + e % m;
      if (y <= x) {
        double v = A[x][y];
#pragma unroll
        for (int k = 0; k < 16; ++k) v = fma(-A[x][k0 + k], A[y][k0 + k], v);
        A[x][y] = v;
      }
    }
    __syncthreads();
  }
  if (w < nb && lane < 16) {   // inverse of diagonal block w: column `lane`
    const int k0 = w * 16;
    double z[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double v = i == lane ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) v = fma(-A[k0 + i][k0 + k], z[k], v);
      z[i] = v / A[k0 + i][k0 + i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Li[k0 + i][k0 + lane] = z[i];
  }
  __syncthreads();
  for (int Ib = 1; Ib < nb; ++Ib) {
    // T = sum_{J <= K < Ib} L[Ib][K] Li[K][J], then Li[Ib][J] = -Li[Ib][Ib] T
    for (int e = tid; e < Ib * 256; e += 256) {
      const int J = e >> 8, r = (e >> 4) & 15, c = e & 15;
      double v = 0.0;
      for (int k = J * 16; k < Ib * 16; ++k) v = fma(A[Ib * 16 + r][k], Li[k][J * 16 + c], v);
      T[Ib * 16 + r][J * 16 + c] = v;
    }
    __syncthreads();
    for (int e = tid; e < Ib * 256; e += 256) {
      const int J = e >> 8, r = (e >> 4) & 15, c = e & 15;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) v = fma(-Li[Ib * 16 + r][Ib * 16 + k], T[Ib * 16 + k][J * 16 + c], v);
      Li[Ib * 16 + r][J * 16 + c] = v;
    }
    __syncthreads();
  }
  // B[k][j] = Li[j][k]
  for (int e = tid; e < nn * nn; e += 256) {
    const int k = e / nn, j = e % nn;
    B[e] = Li[j][k];
  }
}

// Product by G = M M^T without forming G (Remark 4's linear-time top-k
// solvers: the work is linear in the kept entries), for the sampled
// matricization M of the single tail mode (s head rows x MT tail columns),
// on blocks of 32 float64 columns.  First W = M^T X, a wave per tail column
// c: the column's entries (r, v) from the CSC list, lane j of each half
// wave adding v X[r][j] over every second entry (the halves start one entry
// apart), eight entries in flight; the two halves are added.  Loads are
// unconditional at indices clamped into the column, and the extra entries'
// values are zeroed (X is finite).
__global__ __launch_bounds__(256) void k_spmm_cols(const Entry* __restrict__ coo_t,
                                                   const uint32_t* __restrict__ colptr, uint32_t MT,
                                                   FastDiv fMT, const double* __restrict__ X,
                                                   uint32_t ldx, double* __restrict__ W, Status s) {
  if (s.skip()) return;
  const int lane = threadIdx.x & 63, j = lane & 31, half = lane >> 5;
  const uint32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= MT) return;   // the whole wave (no barrier follows)
  const uint32_t e0 = colptr[c], e1 = colptr[c + 1];
  double acc = 0.0;
  if (e1 > e0) {
    for (uint32_t eb = e0 + half; eb < e1; eb += 16) {
      Entry en[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) en[u] = coo_t[min(eb + 2u * u, e1 - 1)];
      double q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = X[(size_t)fMT.div(en[u].l) * ldx + j];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        acc = fma((double)en[u].v * (eb + 2u * u < e1 ? 1.0 : 0.0), q[u], acc);
    }
  }
  acc += __shfl_xor(acc, 32, 64);
  if (half == 0) W[(size_t)c * 32 + j] = acc;
}

// Then C = al M W + be X + ga Xp (the filter epilogue of the products by G,
// columns 0..31, ld ldc), a workgroup per head row r: its entries (c, v)
// from the CSR list, eight groups of 32 lanes taking every eighth entry,
// eight in flight per lane; the group sums are added in group order.
__global__ __launch_bounds__(256) void k_spmm_rows(const Entry* __restrict__ coo_l,
                                                   const uint32_t* __restrict__ rowptr, uint32_t MT,
                                                   const double* __restrict__ W, double* __restrict__ C,
                                                   uint32_t ldc, const double* __restrict__ X, Cheb ch,
                                                   Status s) {
  if (s.skip()) return;
  __shared__ double part[8][32];
  const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
  const uint32_t r = blockIdx.x;
  const uint32_t e0 = rowptr[r], e1 = rowptr[r + 1];
  const uint32_t base = r * MT;
  double acc = 0.0;
  if (e1 > e0) {
    for (uint32_t eb = e0 + g; eb < e1; eb += 64) {
      Entry en[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) en[u] = coo_l[min(eb + 8u * u, e1 - 1)];
      double w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = W[(size_t)(en[u].l - base) * 32 + j];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        acc = fma((double)en[u].v * (eb + 8u * u < e1 ? 1.0 : 0.0), w[u], acc);
    }
  }
  part[g][j] = acc;
  __syncthreads();
  if (threadIdx.x < 32) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += part[q][j];
    const ChebCoef cf = cheb_coef(ch);
    const size_t o = (size_t)r * ldc + j;
    double v = cf.al * t;
    if (cf.be != 0.0) v = fma(cf.be, X[o], v);
    if (cf.ga != 0.0) v = fma(cf.ga, ch.Xp[o], v);
    C[o] = v;
  }
}

// Deterministic start block for the subspace iteration (hash of position).
__global__ void k_ss_init(double* __restrict__ Q, uint32_t ldq, uint32_t M, uint32_t n,
                          const int32_t* tag, int32_t tagval, Status s) {
  if (s.skip() || *tag == tagval) return;
  uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= M * n) return;
  uint32_t i = e / n, j = e % n;
  uint32_t h = i * 0x9E3779B1u ^ (j + 1) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  Q[(size_t)i * ldq + j] = (double)(h >> 8) * (1.0 / 16777216.0) - 0.5;
}

__global__ void k_copy64(const double* __restrict__ src, double* __restrict__ dst, uint32_t n,
                         Status s) {
  if (s.skip()) return;
  uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

// Residuals of the top R Ritz pairs: converged if all
// ||Z2[:,r] - theta_r Qr[:,r]|| <= tol * theta_0; single workgroup.
constexpr int kSsCheckThreads = 512;

__global__ __launch_bounds__(kSsCheckThreads) void k_ss_check(const double* __restrict__ Z2, const double* __restrict__ Qr,
                                                  uint32_t ld, uint32_t M, const double* __restrict__ theta,
                                                  uint32_t R, double tol, double tol_fail, int32_t* done, int last,
                                                  int32_t* stat_it, int32_t it, int32_t* ritz,
                                                  Status s) {
  if (s.skip()) return;
  constexpr int NW = kSsCheckThreads / 64;
  __shared__ double res[16][NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double th[16], acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    th[r] = theta[min((uint32_t)r, R - 1)];
    acc[r] = 0.0;
  }
  // two rows per thread and round, the 16 columns of both blocks loaded
  // unconditionally (columns from R on repeat column R - 1, rows past M
  // repeat row M - 1; their terms are zeroed)
  for (uint32_t m0 = threadIdx.x; m0 < M; m0 += 2 * kSsCheckThreads) {
    double z[2][16], q[2][16];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const size_t row = (size_t)min(m0 + h * kSsCheckThreads, M - 1) * ld;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        z[h][r] = Z2[row + min((uint32_t)r, R - 1)];
        q[h][r] = Qr[row + min((uint32_t)r, R - 1)];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double keep = m0 + h * kSsCheckThreads < M ? 1.0 : 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const double d = (z[h][r] - th[r] * q[h][r]) * keep;
        acc[r] = fma(d, d, acc[r]);
      }
    }
  }
  for (int r = 0; r < 16; ++r) {
    double v = acc[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) res[r][w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double worst = 0.0;
    for (uint32_t r = 0; r < R; ++r) {
      double t = 0.0;
      for (int q = 0; q < NW; ++q) t += res[r][q];
      const double v = sqrt(t);
      worst = v > worst ? v : worst;
    }
    double ref = fabs(theta[0]);
    *ritz = 1;   // theta holds Ritz values from now on (the filter's tau)
    if (worst <= tol * ref) {
      *done = 1;
      *stat_it = it + 1;
    } else if (last) {
      *stat_it = 10000 + it + 1;
      if (worst > tol_fail * ref) atomicCAS(s.st, 0, MACH_ENOCONV);
    }
  }
}

// ---------------------------------------------------------------------------
// Factor update
// ---------------------------------------------------------------------------

// Aw[i][r] = V[i][r] (row-side Gram: the eigenvectors are the factor).
__global__ void k_take_cols(const double* __restrict__ V, uint32_t ldv, uint32_t I, uint32_t R,
                            double* __restrict__ Aw, Status s) {
  if (s.skip()) return;
  uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= I * 16) return;
  uint32_t i = e >> 4, r = e & 15;
  Aw[e] = r < R ? V[(size_t)i * ldv + r] : 0.0;
}

// Column-side Gram of M = Y_(k) (dense float32): Aw[i][r] = sum_j M[i, j] V[j][r] / sqrt(lam_r).
__global__ __launch_bounds__(256) void k_backproject_dense(const float* __restrict__ Y, uint32_t I,
                                                           uint32_t Q, uint32_t J, FastDiv fQ,
                                                           const double* __restrict__ V, uint32_t ldv,
                                                           const double* __restrict__ lam, uint32_t R,
                                                           double* __restrict__ Aw, Status s) {
  if (s.skip()) return;
  uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!(lam[R - 1] > 1e-13 * lam[0])) atomicCAS(s.st, 0, MACH_EDEGENERATE);
  }
  if (i >= I) return;
  double acc[16];
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;
  for (uint32_t j = 0; j < J; ++j) {
    uint32_t q = fQ.div(j);
    double y = (double)Y[(size_t)q * I * Q + (size_t)i * Q + (j - q * Q)];
    const double* v = V + (size_t)j * ldv;
    for (uint32_t r = 0; r < R; ++r) acc[r] = fma(y, v[r], acc[r]);
  }
  for (uint32_t r = 0; r < 16; ++r)
    Aw[(size_t)i * 16 + r] = r < R ? acc[r] / sqrt(fmax(lam[r], 1e-300)) : 0.0;
}

// Same for the sampled unfolding Xhat_(n): element (i, j) at off(j) + i * Q.
__global__ __launch_bounds__(256) void k_backproject_xhat(const uint64_t* __restrict__ bitmap,
                                                          const uint32_t* __restrict__ wrank,
                                                          const Entry* __restrict__ coo, uint32_t I,
                                                          uint32_t Q, uint32_t J, FastDiv fQ,
                                                          const double* __restrict__ V, uint32_t ldv,
                                                          const double* __restrict__ lam, uint32_t R,
                                                          double* __restrict__ Aw, Status s) {
  if (s.skip()) return;
  uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!(lam[R - 1] > 1e-13 * lam[0])) atomicCAS(s.st, 0, MACH_EDEGENERATE);
  }
  if (i >= I) return;
  double acc[16];
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;
  for (uint32_t j = 0; j < J; ++j) {
    uint32_t q = fQ.div(j);
    uint32_t l = q * I * Q + i * Q + (j - q * Q);
    uint64_t word = bitmap[l >> 6];
    uint32_t b = l & 63;
    if (!((word >> b) & 1ull)) continue;
    uint64_t below = b ? (word & ((~0ull) >> (64 - b))) : 0ull;
    double x = (double)coo[wrank[l >> 6] + (uint32_t)__popcll(below)].v;
    const double* v = V + (size_t)j * ldv;
    for (uint32_t r = 0; r < R; ++r) acc[r] = fma(x, v[r], acc[r]);
  }
  for (uint32_t r = 0; r < 16; ++r)
    Aw[(size_t)i * 16 + r] = r < R ? acc[r] / sqrt(fmax(lam[r], 1e-300)) : 0.0;
}

// Column-side Gram of Xhat_(n) when mode n is the only tail mode: row i of
// the matricization is tail column c = i of the column-grouped copy and
// the matricization column of an entry is its head row l / MT.  One wave
// per row: lanes take entries, then a fixed butterfly sums the lanes.
__global__ __launch_bounds__(256) void k_backproject_cols(const Entry* __restrict__ coo_t,
                                                          const uint32_t* __restrict__ colptr,
                                                          uint32_t I, FastDiv fMT,
                                                          const double* __restrict__ V, uint32_t ldv,
                                                          const double* __restrict__ lam, uint32_t R,
                                                          double* __restrict__ Aw, Status s) {
  if (s.skip()) return;
  const int lane = threadIdx.x & 63;
  const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!(lam[R - 1] > 1e-13 * lam[0])) atomicCAS(s.st, 0, MACH_EDEGENERATE);
  }
  double acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;
  if (i < I) {
    // all 16 factor entries of a row are loaded unconditionally (columns
    // from R on repeat column R - 1, inside the row; their sums are unused)
    for (uint32_t e = colptr[i] + lane; e < colptr[i + 1]; e += 64) {
      Entry en = coo_t[e];
      const double* v = V + (size_t)fMT.div(en.l) * ldv;
      double x = (double)en.v;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = fma(x, v[min((uint32_t)r, R - 1)], acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r)
    for (int m = 32; m > 0; m >>= 1) acc[r] += __shfl_xor(acc[r], m, 64);
  if (i < I && lane < 16)
    Aw[(size_t)i * 16 + lane] = (uint32_t)lane < R ? acc[lane] / sqrt(fmax(lam[lane], 1e-300)) : 0.0;
}

// Per-chunk column maxima of |Aw| (value, then lowest row).
__global__ __launch_bounds__(256) void k_colmax_partial(const double* __restrict__ Aw, uint32_t I,
                                                        uint32_t R, uint32_t rows,
                                                        double* __restrict__ pv, uint32_t* __restrict__ pi,
                                                        Status s) {
  if (s.skip()) return;
  __shared__ double bv[256];
  __shared__ uint32_t bi[256];
  uint32_t r = threadIdx.x & 15, g = threadIdx.x >> 4;
  uint32_t i0 = blockIdx.x * rows, i1 = min(I, i0 + rows);
  double best = -1.0;
  uint32_t bidx = 0xffffffffu;
  for (uint32_t i = i0 + g; i < i1; i += 16) {
    double v = fabs(Aw[(size_t)i * 16 + r]);
    if (v > best) {
      best = v;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  if (threadIdx.x < 16) {
    double b = -1.0;
    uint32_t bx = 0xffffffffu;
    for (int gg = 0; gg < 16; ++gg) {
      double v = bv[gg * 16 + threadIdx.x];
      uint32_t ix = bi[gg * 16 + threadIdx.x];
      if (v > b || (v == b && ix < bx)) {
        b = v;
        bx = ix;
      }
    }
    pv[blockIdx.x * 16 + threadIdx.x] = b;
    pi[blockIdx.x * 16 + threadIdx.x] = bx;
  }
}

// Applies the sign rule, writes the float64 factor (I x R) and the float32
// working copy (I x 16, zero padded).
__global__ __launch_bounds__(256) void k_sign_store(const double* __restrict__ Aw, uint32_t I, uint32_t R,
                                                    const double* __restrict__ pv,
                                                    const uint32_t* __restrict__ pi, uint32_t nchunk,
                                                    double* __restrict__ Aout, float* __restrict__ af,
                                                    Status s) {
  if (s.skip()) return;
  __shared__ double sg[16];
  __shared__ double bv[256];
  __shared__ uint32_t bi[256];
  {
    // column r = tid % 16: 16 threads scan the chunk maxima, then one
    // combines them (largest value, lowest row on ties: order-free)
    // (four chunks per round, loaded unconditionally at clamped indices)
    const uint32_t r = threadIdx.x & 15, g = threadIdx.x >> 4;
    double b = -1.0;
    uint32_t bx = 0xffffffffu;
    for (uint32_t c0 = g; c0 < nchunk; c0 += 64) {
      double v[4];
      uint32_t ix[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t c = min(c0 + 16u * u, nchunk - 1);
        v[u] = pv[c * 16 + r];
        ix[u] = pi[c * 16 + r];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (c0 + 16u * u < nchunk && (v[u] > b || (v[u] == b && ix[u] < bx))) {
          b = v[u];
          bx = ix[u];
        }
    }
    bv[threadIdx.x] = b;
    bi[threadIdx.x] = bx;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    double b = -1.0;
    uint32_t bx = 0xffffffffu;
    for (int g = 0; g < 16; ++g) {
      const double v = bv[g * 16 + threadIdx.x];
      const uint32_t ix = bi[g * 16 + threadIdx.x];
      if (v > b || (v == b && ix < bx)) {
        b = v;
        bx = ix;
      }
    }
    double sgn = 1.0;
    if (threadIdx.x < R && bx < I && Aw[(size_t)bx * 16 + threadIdx.x] < 0.0) sgn = -1.0;
    sg[threadIdx.x] = sgn;
  }
  __syncthreads();
  uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= I * 16) return;
  uint32_t i = e >> 4, r = e & 15;
  double v = r < R ? sg[r] * Aw[e] : 0.0;
  if (r < R) Aout[(size_t)i * R + r] = v;
  af[e] = (float)v;
}

// fit = 1 - sqrt(max(0, ||Xhat||^2 - ||G||^2)) / ||Xhat||, with
// ||G||^2 = sum of the top R eigenvalues of the last mode's Gram / p^2.
__global__ void k_fit(const double* __restrict__ lam, uint32_t R, const SampleHdr* hdr,
                      const int32_t* st, double* fit, double* core2_out) {
  if (hdr->status != 0 || *st != 0) return;
  double p2 = hdr->p * hdr->p;
  double g2 = 0.0;
  for (uint32_t r = 0; r < R; ++r) g2 += lam[r];
  g2 /= p2;
  double x2 = hdr->sumsq / p2;
  if (fit) *fit = 1.0 - sqrt(fmax(0.0, x2 - g2)) / sqrt(x2);
  if (core2_out) *core2_out = g2;
}

// G[(q*O + o)*R + r] = (1/p) sum_i A[i][r] Y[(o*I + i)*Q + q]; one
// workgroup per core entry, fixed-order tree over i.
__global__ __launch_bounds__(256) void k_core(const float* __restrict__ Y, uint32_t O, uint32_t I,
                                              uint32_t Q, const double* __restrict__ A, uint32_t R,
                                              double* __restrict__ G, const SampleHdr* hdr,
                                              const int32_t* st) {
  if (hdr->status != 0 || *st != 0) return;
  __shared__ double red[2][4];
  uint32_t e = blockIdx.x;
  uint32_t r = e % R, t = e / R;
  uint32_t o = t % O, q = t / O;
  double acc = 0.0, dummy = 0.0;
  for (uint32_t i = threadIdx.x; i < I; i += 256)
    acc = fma(A[(size_t)i * R + r], (double)Y[((size_t)o * I + i) * Q + q], acc);
  block_sum2(acc, dummy, red);
  if (threadIdx.x == 0) G[e] = acc / hdr->p;
}

// G[q * MT + c] = TT[c * KH + q] / p: the core of a Tucker-n decomposition
// whose single tail mode is uncompressed (C order R_1 x .. x R_h x MT).
__global__ __launch_bounds__(256) void k_core_ident(const float* __restrict__ TT, uint32_t MT, uint32_t KH,
                                                    double* __restrict__ G, const SampleHdr* hdr,
                                                    const int32_t* st) {
  if (hdr->status != 0 || *st != 0) return;
  const uint32_t e = blockIdx.x * 256 + threadIdx.x;
  if (e >= MT * KH) return;
  const uint32_t q = e / MT, c = e - q * MT;
  G[e] = (double)TT[(size_t)c * KH + q] / hdr->p;
}

__global__ __launch_bounds__(256) void k_norm2(const double* __restrict__ G, uint32_t n, double* out,
                                               const SampleHdr* hdr, const int32_t* st) {
  if (hdr->status != 0 || *st != 0) return;
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (uint32_t e = threadIdx.x; e < n; e += 256) a += G[e] * G[e];
  block_sum2(a, b, red);
  if (threadIdx.x == 0) *out = a;
}

// Clears the status word, the warm-start tags and the per-mode solve
// statistics (status words 24..39: sweep solves, then HOSVD solves).
__global__ void k_solver_init(int32_t* st, int32_t* tags, int ntags) {
  int t = threadIdx.x;
  if (t == 0) *st = 0;
  if (t < ntags) tags[t] = 0;
  if (t < 16) st[24 + t] = 0;
}

}  // namespace
}  // namespace mach

namespace mach {
namespace {

struct Ctx {
  const SolverLayout* SL;
  char* ws;
  const SampleHdr* hdr;
  hipStream_t st;
  int32_t* status() const { return (int32_t*)(ws + SL->status); }
  int32_t* tags() const { return (int32_t*)(ws + SL->tags); }
  Status stat(bool with_done = false) const {
    Status s;
    s.hdr = hdr;
    s.st = status();
    s.done = with_done ? tags() + kTagDone : nullptr;
    return s;
  }
  double* d(size_t off) const { return (double*)(ws + off); }
};

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

__global__ void k_set_int(int32_t* p, int32_t v) {
  if (threadIdx.x == 0) *p = v;
}

void gemm(const Ctx& c, const double* A, uint32_t lda, const double* B, uint32_t ldb, double* C,
          uint32_t ldc, uint32_t M, uint32_t K, uint32_t N, bool with_done) {
  hipLaunchKernelGGL(k_gemm64, dim3(cdiv(M, 16)), dim3(256), 0, c.st, A, lda, B, ldb, C, ldc, M, K,
                     N, c.stat(with_done));
}

// C (s x 64, ld kBlock) = G (s x s) * X (s x n, ld kBlock): split over the
// summation index when it is long, so that every CU gets a tile.
void gemm_sq(const Ctx& c, const double* G, uint32_t s, const double* X, double* C, uint32_t n,
             bool with_done, Cheb ch = Cheb{0, nullptr, 0, nullptr, nullptr}) {
  const uint32_t nks = s >= 512 ? cdiv(s, kSplitK) : 1;
  // one slice: the kernel's partial layout (rows of 64) is C itself
  double* P = nks > 1 ? c.d(c.SL->skpart) : C;
  if (n <= 32)
    hipLaunchKernelGGL(k_gemm_splitk<32>, dim3(cdiv(s, 64), nks), dim3(256), 0, c.st, G, s, X, kBlock, P,
                       s, s, n, ch, c.stat(with_done));
  else
    hipLaunchKernelGGL(k_gemm_splitk<64>, dim3(cdiv(s, 64), nks), dim3(256), 0, c.st, G, s, X, kBlock, P,
                       s, s, n, ch, c.stat(with_done));
  if (nks > 1)
    hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv((uint64_t)s * 64, 256)), dim3(256), 0, c.st, P, nks,
                       s, C, kBlock, X, ch, c.stat(with_done));
}

// The operator of the subspace iteration: a formed s x s Gram G, or (G
// null) M M^T applied through the sparse layouts without forming it.
struct SsOp {
  const double* G;
  const Entry* coo_l;
  const uint32_t* rowptr;
  const Entry* coo_t;
  const uint32_t* colptr;
  uint32_t MT;
  FastDiv fMT;
  double* W;   // MT x 32 float64
};

// C = op(X) through the filter epilogue (n columns; the sparse form takes
// blocks of exactly 32).
void apply_op(const Ctx& c, const SsOp& op, uint32_t s, const double* X, double* C, uint32_t n,
              bool with_done, Cheb ch = Cheb{0, nullptr, 0, nullptr, nullptr}) {
  if (op.G) {
    gemm_sq(c, op.G, s, X, C, n, with_done, ch);
    return;
  }
  hipLaunchKernelGGL(k_spmm_cols, dim3(cdiv(op.MT, 4)), dim3(256), 0, c.st, op.coo_t, op.colptr, op.MT,
                     op.fMT, X, kBlock, op.W, c.stat(with_done));
  hipLaunchKernelGGL(k_spmm_rows, dim3(s), dim3(256), 0, c.st, op.coo_l, op.rowptr, op.MT, op.W, C,
                     kBlock, X, ch, c.stat(with_done));
}

void jacobi(const Ctx& c, const double* G, uint32_t nchunk, uint32_t n, double* V, double* lam,
            int32_t* tag, int32_t tagval, bool with_done, int rtop, double tol2 = kOffTol2) {
  JacArgs a;
  a.G = G;
  a.nchunk = nchunk;
  a.n = n;
  a.V = V;
  a.lam = lam;
  a.tag = tag;
  a.tagval = tagval;
  a.rtop = rtop;
  a.tol2 = tol2;
  a.s = c.stat(with_done);
  if (n <= 16)
    hipLaunchKernelGGL((k_jacobi_small<16, 256>), dim3(1), dim3(256), 0, c.st, a);
  else if (n <= 32)
    hipLaunchKernelGGL((k_jacobi_small<32, 512>), dim3(1), dim3(512), 0, c.st, a);
  else
    hipLaunchKernelGGL((k_jacobi_small<64, 1024>), dim3(1), dim3(1024), 0, c.st, a);
}

// Cholesky-QR of X (M x n, ld kBlock): `passes` passes (the first shifted
// by 1e-15 tr(S) / n), alternating between X and the scratch Y.  Returns
// the buffer holding the result (X after an even number of passes).
// The n x n partials (chunk-minor, nchunk chunks) summed into one copy in
// the reduction scratch, one wave per entry, so that the single-workgroup
// kernel after it reads n^2 values instead of n^2 nchunk.
const double* reduce_square(const Ctx& c, const double* part, uint32_t nchunk, uint32_t n,
                            Status sd) {
  ReduceArgs r{};
  r.in = part;
  r.out = c.d(c.SL->sred) + kSredGram;
  r.nent = n * n;
  r.gsize = r.nent;
  r.es = nchunk;
  r.cs = 1;
  r.nch[0] = nchunk;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(cdiv(r.nent, 4)), dim3(256), 0, c.st, r, sd);
  return r.out;
}

double* orthonormalise(const Ctx& c, double* X, double* Y, uint32_t M, uint32_t n, int passes,
                       bool with_done) {
  Status sd = c.stat(with_done);
  uint32_t nchunk = cdiv(M, 32);
  if (nchunk > 64) nchunk = 64;
  uint32_t rows = cdiv(M, nchunk);
  nchunk = cdiv(M, rows);
  double* B = c.d(c.SL->H);
  double* src = X;
  double* dst = Y;
  for (int pass = 0; pass < passes; ++pass) {
    hipLaunchKernelGGL(k_atb_partial, dim3(nchunk), dim3(256), 0, c.st, src, kBlock, src, kBlock, M, n,
                       rows, c.d(c.SL->part), sd);
    const double* S = nchunk > 1 ? reduce_square(c, c.d(c.SL->part), nchunk, n, sd) : c.d(c.SL->part);
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, c.st, S, 1u, n, pass == 0 ? 1e-15 : 0.0, B,
                       sd);
    gemm(c, src, kBlock, B, n, dst, kBlock, M, n, n, with_done);
    double* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Top eigenpairs of the s x s matrix G (s > 64) by block subspace iteration
// on b = min(64, max(32, 2R rounded up to 16)) columns: the block is
// multiplied by G every step and re-orthonormalised (one Cholesky-QR pass)
// after every second step; every 8 steps and at the end, Rayleigh-Ritz on
// the orthonormalised block (Jacobi on b x b), and the iteration stops once
// the top R Ritz residuals are below 1e-10 of the largest Ritz value (the
// remaining steps are skipped on the device).  Q (s x 64, ld 64) holds the
// start block (warm start if *tag == tagval); on return its first R columns
// are the Ritz vectors and lam the Ritz values, descending.
void subspace_topk(const Ctx& c, const SsOp& op, uint32_t s, uint32_t R, double* Q, double* lam,
                   int32_t* tag, int32_t tagval, int maxit, int32_t* stat_it,
                   SolveTol tol = solve_tol(MACH_F32)) {
  uint32_t b = 2 * R;
  b = b < 32 ? 32 : (b + 15) / 16 * 16;
  if (b > kBlock) b = kBlock;
  if (b > s) b = s;
  int32_t* tags = c.tags();
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c.st, tags + kTagDone, 0);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c.st, tags + kTagRitz, 0);
  hipLaunchKernelGGL(k_ss_init, dim3(cdiv((uint64_t)s * b, 256)), dim3(256), 0, c.st, Q, kBlock, s,
                     b, tag, tagval, c.stat());
  // Buffers: the Ritz vectors of every Rayleigh-Ritz step go to Qr (so the
  // converged ones stay there when later steps are skipped); the block and
  // its products rotate through Q, Z and Z2.
  double* Qr = c.d(c.SL->Qrs);
  double* H = c.d(c.SL->part);
  double* VH = c.d(c.SL->VH);
  double* lamH = c.d(c.SL->lamH);
  double* pool[3] = {Q, c.d(c.SL->Zs), c.d(c.SL->Z2s)};
  auto other = [&](const double* a, const double* b2) {
    for (double* p : pool)
      if (p != a && p != b2) return p;
    return pool[0];
  };
  double* cur = orthonormalise(c, Q, other(Q, nullptr), s, b, 2, false);
  Status sd = c.stat(true);
  double* xpair = nullptr;   // input of the current pair of filter steps
  for (int it = 0; it < maxit; ++it) {
    const bool last = it == maxit - 1;
    const bool rr = (it % 8 == 7) || last;
    // steps come in pairs (a degree-2 Chebyshev filter once Ritz values
    // exist, plain products before), orthonormalised after the second
    Cheb ch{it % 2 == 0 ? 1 : 2, lamH, b - 1, tags + kTagRitz, nullptr};
    double* z;
    if (it % 2 == 0) {
      xpair = cur;
      z = other(cur, nullptr);
    } else {
      ch.Xp = xpair;
      z = other(cur, xpair);
    }
    apply_op(c, op, s, cur, z, b, true, ch);
    if (!rr) {
      if (it % 2 == 1) z = orthonormalise(c, z, other(z, nullptr), s, b, 1, true);
      cur = z;
      continue;
    }
    double* w = other(z, nullptr);
    z = orthonormalise(c, z, w, s, b, 2, true);   // result back in z
    w = other(z, nullptr);
    apply_op(c, op, s, z, w, b, true);             // w = G z
    uint32_t nchunk = cdiv(s, 32);
    if (nchunk > 64) nchunk = 64;
    uint32_t rows = cdiv(s, nchunk);
    nchunk = cdiv(s, rows);
    hipLaunchKernelGGL(k_atb_partial, dim3(nchunk), dim3(256), 0, c.st, z, kBlock, w, kBlock, s, b, rows,
                       H, sd);
    const double* Hs = nchunk > 1 ? reduce_square(c, H, nchunk, b, sd) : H;
    // The block is the previous Ritz vectors times G^8, orthonormalised in
    // column order, so H is close to diagonal as it stands: start from the
    // identity (the previous step's rotation would undo that).
    jacobi(c, Hs, 1, b, VH, lamH, tags + kTagRR, 0, true, (int)R, 1e-24);
    double* zr = other(z, w);
    gemm(c, z, kBlock, VH, b, Qr, kBlock, s, b, b, true);
    gemm(c, w, kBlock, VH, b, zr, kBlock, s, b, b, true);
    hipLaunchKernelGGL(k_ss_check, dim3(1), dim3(kSsCheckThreads), 0, c.st, zr, Qr, kBlock, s, lamH, R, tol.res, tol.res_fail,
                       tags + kTagDone, last ? 1 : 0, stat_it, it, tags + kTagRitz, c.stat(true));
    cur = Qr;
  }
  hipLaunchKernelGGL(k_copy64, dim3(cdiv((uint64_t)s * kBlock, 256)), dim3(256), 0, c.st, Qr, Q,
                     s * kBlock, c.stat());
  hipLaunchKernelGGL(k_copy64, dim3(1), dim3(256), 0, c.st, lamH, lam, b, c.stat());
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c.st, tag, tagval);
}

__global__ __launch_bounds__(256) void k_ata16_partial(const double* __restrict__ Aw, uint32_t I,
                                                       double* __restrict__ part, Status s) {
  if (s.skip()) return;
  __shared__ double rows[256][17];
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const double x = Aw[(size_t)min(i, I - 1) * 16 + r];   // unconditional load
    rows[threadIdx.x][r] = i < I ? x : 0.0;
  }
  __syncthreads();
  const int x = threadIdx.x >> 4, y = threadIdx.x & 15;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
  for (int t = 0; t < 256; t += 4) {
    g0 = fma(rows[t][x], rows[t][y], g0);
    g1 = fma(rows[t + 1][x], rows[t + 1][y], g1);
    g2 = fma(rows[t + 2][x], rows[t + 2][y], g2);
    g3 = fma(rows[t + 3][x], rows[t + 3][y], g3);
  }
  part[(size_t)blockIdx.x * 256 + threadIdx.x] = (g0 + g1) + (g2 + g3);
}

// The 16 x 16 Gram of a tall factor from its per-workgroup partials
// (chunk-major, 256 entries each): summed into sred once when there are
// several, so that every workgroup of the apply step reads one copy.
const double* reduce_tall(const Ctx& c, const double* part, uint32_t nwg) {
  if (nwg <= 1) return part;
  ReduceArgs r{};
  r.in = part;
  r.out = c.d(c.SL->sred) + kSredTall;
  r.nent = 256;
  r.gsize = 256;
  r.es = 1;
  r.cs = 256;
  r.nch[0] = nwg;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(64), dim3(256), 0, c.st, r, c.stat());
  return r.out;
}

// Aw (I x 16, nearly orthonormal columns) -> one Cholesky-QR pass, the sign
// rule, and the float64 / float32 stores.
void finish_factor(const Ctx& c, uint32_t I, uint32_t R, double* Aout, float* af) {
  uint32_t nwg = cdiv(I, 256);
  double* part = c.d(c.SL->part);
  hipLaunchKernelGGL(k_ata16_partial, dim3(nwg), dim3(256), 0, c.st, c.d(c.SL->Aw), I, part, c.stat());
  const double* g16 = reduce_tall(c, part, nwg);
  hipLaunchKernelGGL(k_chol_apply_tall, dim3(nwg), dim3(256), 0, c.st, c.d(c.SL->Aw), I, R, g16, 1u,
                     c.d(c.SL->pv), (uint32_t*)(c.ws + c.SL->pi), c.stat());
  hipLaunchKernelGGL(k_sign_store, dim3(cdiv((uint64_t)I * 16, 256)), dim3(256), 0, c.st, c.d(c.SL->Aw),
                     I, R, c.d(c.SL->pv), (const uint32_t*)(c.ws + c.SL->pi), nwg, Aout, af, c.stat());
}

// Sign rule and stores from Aw (I x 16 float64).
void sign_store(const Ctx& c, uint32_t I, uint32_t R, double* Aout, float* af) {
  uint32_t nchunk = cdiv(I, 256);
  if (nchunk > 1024) nchunk = 1024;
  uint32_t rows = cdiv(I, nchunk);
  double* pv = c.d(c.SL->pv);
  uint32_t* pi = (uint32_t*)(c.ws + c.SL->pi);
  hipLaunchKernelGGL(k_colmax_partial, dim3(nchunk), dim3(256), 0, c.st, c.d(c.SL->Aw), I, R, rows, pv,
                     pi, c.stat());
  hipLaunchKernelGGL(k_sign_store, dim3(cdiv((uint64_t)I * 16, 256)), dim3(256), 0, c.st,
                     c.d(c.SL->Aw), I, R, pv, pi, nchunk, Aout, af, c.stat());
}

}  // namespace

hipError_t launch_solver_init(const SolverLayout& SL, char* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_solver_init, dim3(1), dim3(64), 0, st, (int32_t*)(ws + SL.status),
                     (int32_t*)(ws + SL.tags), 16);
  if (SL.laneb[15])
    hipLaunchKernelGGL(k_solver_init, dim3(1), dim3(64), 0, st, (int32_t*)(ws + SL.status),
                       (int32_t*)(ws + SL.laneb[15]), 16);
  return hipGetLastError();
}

hipError_t launch_mode_update(const ShapeInfo& si, const SolverLayout& SL, char* ws, int k,
                              double* A_out, int prec, const SampleHdr* hdr, hipStream_t st) {
  Ctx c{&SL, ws, hdr, st};
  const ModePlan& m = SL.mp[k];
  const SolveTol tol = solve_tol(prec);
  int32_t tagval = 0x4d000000 | (k << 16) | (int32_t)m.s;
  if (m.kside && m.I <= (uint32_t)kSsMaxI && m.K >= (uint32_t)kSsB && m.K <= (uint32_t)kSsMaxK &&
      m.R <= 8) {
    SsArgs a;
    a.Y = (const float*)(ws + m.ybuf);
    a.O = m.O;
    a.I = m.I;
    a.Q = m.Q;
    a.K = m.K;
    a.R = m.R;
    a.Aprev = A_out;
    a.state = c.d(m.V);
    a.lam = c.d(m.lam);
    a.tag = c.tags() + k;
    a.tagval = tagval;
    a.Aout = A_out;
    a.af = (float*)(ws + SL.af[k]);
    a.stats = (int32_t*)(ws + SL.status + 96) + k;
    a.rtol = tol.res;
    a.rfail = tol.res_fail;
    a.st = c.stat();
    hipLaunchKernelGGL((k_mode_ss<256, 0>), dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
  }
  if (m.s <= (uint32_t)kSmallEig) {
    uint32_t nchunk = 1;
    hipError_t e = launch_gram_y_partials(SL, ws, k, prec, hdr, st, &nchunk);
    if (e != hipSuccess) return e;
    SolveArgs a;
    a.part = c.d(SL.Gpart);
    a.ctc = nullptr;
    a.cstride = kCtcChunks;
    a.nother = 0;
    ReduceArgs rctc{};
    if (m.kside) {
      CtcArgs ca{};
      for (int j = 0; j < si.d; ++j) {
        if (j == k) continue;
        ca.old[ca.n] = (const float*)(ws + m.snap[j]);
        ca.cur[ca.n] = (const float*)(ws + SL.af[j]);
        ca.I[ca.n] = si.dims[j];
        ca.nch[ca.n] = ctc_chunks(si.dims[j]);
        a.onch[ca.n] = ca.nch[ca.n];
        a.oR[ca.n] = SL.mp[j].R;
        a.ost[ca.n] = m.kst[j];
        ++ca.n;
      }
      a.nother = ca.n;
      hipLaunchKernelGGL(k_ctc_partial, dim3(kCtcChunks, ca.n), dim3(256), 0, st, ca, c.d(SL.part),
                         c.stat());
      // C_j of every other mode summed once (one wave per entry), in the
      // same launch as the Gram partials' sums below when there are any
      ReduceArgs r{};
      r.in = c.d(SL.part);
      r.out = c.d(SL.sred) + kSredCtc;
      r.nent = 256 * ca.n;
      r.gsize = 256;
      r.es = kCtcChunks;
      r.cs = 1;
      for (int j = 0; j < ca.n; ++j) {
        r.nch[j] = ca.nch[j];
        a.onch[j] = 1;
      }
      rctc = r;
      a.ctc = r.out;
      a.cstride = 1;
    }
    ReduceArgs rg{};
    if (nchunk > 1) {   // the Gram partials likewise
      rg.in = c.d(SL.Gpart);
      rg.out = c.d(SL.sred) + kSredGram;
      rg.nent = m.s * m.s;
      rg.gsize = rg.nent;
      rg.es = nchunk;
      rg.cs = 1;
      rg.nch[0] = nchunk;
      a.part = rg.out;
      nchunk = 1;
    }
    if (rctc.nent && rg.nent)
      hipLaunchKernelGGL(k_reduce_chunks2, dim3(cdiv(rctc.nent + rg.nent, 4)), dim3(256), 0, st, rctc, rg,
                         c.stat());
    else if (rctc.nent || rg.nent)
      hipLaunchKernelGGL(k_reduce_chunks, dim3(cdiv(rctc.nent + rg.nent, 4)), dim3(256), 0, st,
                         rctc.nent ? rctc : rg, c.stat());
    a.nchunk = nchunk;
    a.s = m.s;
    a.I = m.I;
    a.R = m.R;
    a.kside = m.kside;

    a.V = c.d(m.V);
    a.lam = c.d(m.lam);
    a.tag = c.tags() + k;
    a.tagval = tagval;
    a.M = c.d(SL.small);
    a.Aout = A_out;
    a.af = (float*)(ws + SL.af[k]);
    a.stats = (int32_t*)(ws + SL.status + 96) + k;
    a.tol2 = tol.off2;
    a.st = c.stat();
    // Row-side Gram of side 33..64 and R <= 12: block iteration on the Gram
    // first (its own warm-start tag); the Jacobi solve runs, cold, only
    // when that did not pass its test.
    if (!m.kside && m.s > 32 && m.s <= (uint32_t)kSsMaxK && m.R <= 12) {
      SsArgs g{};
      g.G = a.part;
      g.done = c.tags() + kTagDone;
      g.I = m.I;
      g.K = m.I;
      g.R = m.R;
      g.Aprev = A_out;
      g.state = c.d(m.V);
      g.lam = c.d(m.lam);
      g.tag = c.tags() + k;
      g.tagval = (tagval & 0x00ffffff) | 0x4e000000;
      g.Aout = A_out;
      g.af = (float*)(ws + SL.af[k]);
      g.stats = a.stats;
      g.rtol = tol.res;
      g.rfail = tol.res_fail;
      g.st = c.stat();
      hipLaunchKernelGGL((k_mode_ss<256, 1>), dim3(1), dim3(256), 0, st, g);
      a.st = c.stat(true);
    }
    if (m.s <= 16)
      hipLaunchKernelGGL((k_mode_solve<16, 256>), dim3(1), dim3(256), 0, st, a);
    else if (m.s <= 32)
      hipLaunchKernelGGL((k_mode_solve<32, 512>), dim3(1), dim3(512), 0, st, a);
    else
      hipLaunchKernelGGL((k_mode_solve<64, 1024>), dim3(1), dim3(1024), 0, st, a);
    if (m.kside) {
      SnapArgs sa{};
      uint32_t nmax = 1;
      for (int j = 0; j < si.d; ++j) {
        if (j == k) continue;
        sa.src[sa.n] = (const float4*)(ws + SL.af[j]);
        sa.dst[sa.n] = (float4*)(ws + m.snap[j]);
        sa.n4[sa.n] = si.dims[j] * 4;
        nmax = std::max(nmax, sa.n4[sa.n]);
        ++sa.n;
      }
      uint32_t nwg = cdiv(m.I, 256);
      double* part = c.d(SL.part);
      // the back-projection, with the snapshot in extra workgroups
      const uint32_t snap_wg = cdiv(nmax, 256);
      hipLaunchKernelGGL(k_bp_tall, dim3(nwg + snap_wg * (uint32_t)sa.n), dim3(256), 0, st,
                         (const float*)(ws + m.ybuf), m.O, m.I, m.Q, c.d(SL.small), m.R, c.d(SL.Aw),
                         part, nwg, sa, snap_wg, c.stat());
      const double* g16 = reduce_tall(c, part, nwg);
      hipLaunchKernelGGL(k_chol_apply_tall, dim3(nwg), dim3(256), 0, st, c.d(SL.Aw), m.I, m.R, g16, 1u,
                         c.d(SL.pv), (uint32_t*)(ws + SL.pi), c.stat());
      hipLaunchKernelGGL(k_sign_store, dim3(cdiv((uint64_t)m.I * 16, 256)), dim3(256), 0, st,
                         c.d(SL.Aw), m.I, m.R, c.d(SL.pv), (const uint32_t*)(ws + SL.pi), nwg, A_out,
                         (float*)(ws + SL.af[k]), c.stat());
    }
    return hipGetLastError();
  }
  hipError_t e = launch_gram_y(SL, ws, k, prec, hdr, st);
  if (e != hipSuccess) return e;
  // Row-side Gram of side 80..256 (a multiple of 16) and R <= 12: block
  // iteration with G read from global memory.
  if (!m.kside && m.s <= (uint32_t)kSsMaxIG && m.s % 16 == 0 && m.R <= 12) {
    SsArgs g{};
    g.G = c.d(SL.G);
    g.I = m.I;
    g.K = m.I;
    g.R = m.R;
    g.Aprev = A_out;
    g.state = c.d(m.Q64);
    g.lam = c.d(m.lam);
    g.tag = c.tags() + k;
    g.tagval = (tagval & 0x00ffffff) | 0x4e000000;
    g.Aout = A_out;
    g.af = (float*)(ws + SL.af[k]);
    g.stats = (int32_t*)(ws + SL.status + 96) + k;
    g.rtol = tol.res;
    g.rfail = tol.res_fail;
    g.st = c.stat();
    hipLaunchKernelGGL((k_mode_ss<256, 2>), dim3(1), dim3(256), 0, st, g);
    return hipGetLastError();
  }
  const double* G = c.d(SL.G);
  double* V = c.d(m.Q64);
  const uint32_t ldv = kBlock;
  subspace_topk(c, SsOp{G}, m.s, m.R, V, c.d(m.lam), c.tags() + k, tagval, 24,
                (int32_t*)(ws + SL.status + 96) + k, tol);
  if (m.kside) {
    uint32_t J = m.O * m.Q;
    hipLaunchKernelGGL(k_backproject_dense, dim3(cdiv(m.I, 256)), dim3(256), 0, st,
                       (const float*)(ws + m.ybuf), m.I, m.Q, J, make_fastdiv(m.Q), V, ldv,
                       c.d(m.lam), m.R, c.d(SL.Aw), c.stat());
    finish_factor(c, m.I, m.R, A_out, (float*)(ws + SL.af[k]));
    return hipGetLastError();
  } else {
    hipLaunchKernelGGL(k_take_cols, dim3(cdiv((uint64_t)m.I * 16, 256)), dim3(256), 0, st, V, ldv,
                       m.I, m.R, c.d(SL.Aw), c.stat());
  }
  sign_store(c, m.I, m.R, A_out, (float*)(ws + SL.af[k]));
  return hipGetLastError();
}

hipError_t launch_hosvd_mode(const ShapeInfo& si, const SparsePtrs& sp, const SolverLayout& SL,
                             char* ws, int n, int R, double* A_out, hipStream_t st) {
  Ctx c{&SL, ws, sp.hdr, st};
  // the single tail mode beyond the sparse Gram's head rows: no Gram, the
  // subspace iteration applies M M^T through the sparse layouts (blocks of
  // 2R <= 32 columns)
  const bool gram_free = SL.hosvd_gram_free && n == si.d - 1;
  if (gram_free && 2 * R > 32) return hipErrorInvalidValue;
  hipError_t e = gram_free ? hipSuccess
                 : sparse_tail_gram_ok(si, SL, n) ? launch_gram_tail_sparse(si, sp, SL, ws, st)
                                                  : launch_gram_xhat(si, sp, SL, ws, n, st);
  if (e != hipSuccess) return e;
  const uint32_t s = SL.hosvd_s[n];
  const double* G = c.d(SL.G);
  const SsOp op = gram_free ? SsOp{nullptr, sp.coo_l, sp.rowptr, sp.coo_t, sp.colptr, si.MT, si.fMT,
                                   c.d(SL.gfw)}
                            : SsOp{G};
  double* V = c.d(SL.Qhs);
  double* lam = c.d(SL.lamH) ;
  uint32_t ldv;
  int32_t* tagc = c.tags() + kTagCold;
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, tagc, 0);
  // Row-side Gram of side 80..256 (a multiple of 16) and R <= 12: block
  // subspace iteration from fixed pseudo-random columns, G read from L2.
  if (!SL.hosvd_kside[n] && s > (uint32_t)kSmallEig && s <= (uint32_t)kSsMaxIG && s % 16 == 0 && R <= 12) {
    SsArgs g{};
    g.G = G;
    g.I = s;
    g.K = s;
    g.R = (uint32_t)R;
    g.Aprev = nullptr;
    g.state = c.d(SL.Aw);
    g.lam = lam;
    g.tag = tagc;
    g.tagval = 0x4f000000 | (int32_t)s;
    g.Aout = A_out;
    g.af = (float*)(ws + SL.af[n]);
    g.stats = (int32_t*)(ws + SL.status + 128) + n;
    g.rtol = solve_tol(MACH_F32).res;
    g.rfail = solve_tol(MACH_F32).res_fail;
    g.st = c.stat();
    hipLaunchKernelGGL((k_mode_ss<256, 2>), dim3(1), dim3(256), 0, st, g);
    return hipGetLastError();
  }
  if (s <= (uint32_t)kSmallEig) {
    ldv = s;
    jacobi(c, G, 1, s, V, lam, tagc, 0x48000000 | (int32_t)s, false, R);
  } else {
    ldv = kBlock;
    subspace_topk(c, op, s, (uint32_t)R, V, lam, tagc, 0x48000000 | (int32_t)s, 48,
                  (int32_t*)(ws + SL.status + 128) + n);
  }
  const uint32_t I = si.dims[n];
  if (SL.hosvd_kside[n] && n == si.d - 1 && si.h == si.d - 1) {
    hipLaunchKernelGGL(k_backproject_cols, dim3(cdiv(I, 4)), dim3(256), 0, st, sp.coo_t, sp.colptr, I,
                       si.fMT, V, ldv, lam, (uint32_t)R, c.d(SL.Aw), c.stat());
    finish_factor(c, I, (uint32_t)R, A_out, (float*)(ws + SL.af[n]));
    return hipGetLastError();
  } else if (SL.hosvd_kside[n]) {
    uint32_t J = si.N / I;
    hipLaunchKernelGGL(k_backproject_xhat, dim3(cdiv(I, 256)), dim3(256), 0, st, sp.bitmap, sp.wrank,
                       sp.coo_l, I, si.stride[n], J, si.fstride[n], V, ldv, lam, (uint32_t)R,
                       c.d(SL.Aw), c.stat());
    finish_factor(c, I, (uint32_t)R, A_out, (float*)(ws + SL.af[n]));
    return hipGetLastError();
  } else {
    hipLaunchKernelGGL(k_take_cols, dim3(cdiv((uint64_t)I * 16, 256)), dim3(256), 0, st, V, ldv, I,
                       (uint32_t)R, c.d(SL.Aw), c.stat());
  }
  sign_store(c, I, (uint32_t)R, A_out, (float*)(ws + SL.af[n]));
  return hipGetLastError();
}

hipError_t launch_fit(const SolverLayout& SL, char* ws, int k, const SampleHdr* hdr, double* fit,
                      hipStream_t st) {
  const ModePlan& m = SL.mp[k];
  hipLaunchKernelGGL(k_fit, dim3(1), dim3(64), 0, st, (const double*)(ws + m.lam), m.R, hdr,
                     (const int32_t*)(ws + SL.status), fit, (double*)(ws + SL.status + 192));
  return hipGetLastError();
}

hipError_t launch_core(const ShapeInfo& si, const SolverLayout& SL, char* ws, const double* A_last,
                       double* G, double* norm2, const SampleHdr* hdr, hipStream_t st) {
  const ModePlan& m = SL.mp[si.d - 1];
  if (SL.ident_last) {   // the last mode uncompressed: G is TT transposed, times 1/p
    const uint32_t n = SL.KH * si.MT;
    const int32_t* stp = (const int32_t*)(ws + SL.status);
    hipLaunchKernelGGL(k_core_ident, dim3(cdiv(n, 256)), dim3(256), 0, st, (const float*)(ws + SL.TT),
                       si.MT, SL.KH, G, hdr, stp);
    if (norm2) hipLaunchKernelGGL(k_norm2, dim3(1), dim3(256), 0, st, G, n, norm2, hdr, stp);
    return hipGetLastError();
  }
  uint32_t n = m.O * m.Q * m.R;
  const int32_t* stp = (const int32_t*)(ws + SL.status);
  hipLaunchKernelGGL(k_core, dim3(n), dim3(256), 0, st, (const float*)(ws + m.ybuf), m.O,
                     m.I, m.Q, A_last, m.R, G, hdr, stp);
  if (norm2)
    hipLaunchKernelGGL(k_norm2, dim3(1), dim3(256), 0, st, G, n, norm2, hdr, stp);
  return hipGetLastError();
}

}  // namespace mach
