// Batched dense LU with partial pivoting and multi-right-hand-side solves.
//
// The local saddle-point blocks A_i = R_i K R_i^T of section 2.1 are
// indefinite (zero pressure block), so they are factored with row pivoting:
// P A = L U, L unit lower, U upper, stored in place, column-major, leading
// dimension = order.  Pivot rows follow the LAPACK convention (ipiv[j] = row
// swapped with row j at step j); ties in the pivot search go to the lowest row.
//
// Right-looking blocked algorithm with two-level blocking, one launch per
// phase for the whole (uneven) batch.  Each outer step covers 2*NB columns:
//   panel  : factor sub-panel 1, A[k:n, k:k+NB] (one workgroup per matrix,
//            rows held in registers and labelled with their interchanged
//            position; DPP wave reductions find the pivot);
//   inner  : its interchanges and U on sub-panel 2's columns, then the rank-NB
//            MFMA update of sub-panel 2; factor sub-panel 2;
//   outer  : the step's interchanges on all other columns, U12 = L11^{-1} A12
//            (one thread per column), A22 -= L21 U12 with MFMA (16x16x4, FP64
//            or FP32), 64x64 tiles, inner dimension 2*NB.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace gdsw {

namespace {

// 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result
// register q of lane l holds D[row(l / 16, q)][l % 16].  The row map differs
// between the FP64 and FP32 instructions (measured on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int q) { return lk + 4 * q; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * lk + q; }
};

constexpr int TILE = 64;
// Tallest panel held in registers: 1024 threads x 2 rows (FP64) or 512 x 6 (FP32).
template <typename T> constexpr int panel_reg_rows() { return sizeof(T) == 8 ? 1024 * 2 : 512 * 6; }

// C[M x N] -= A[M x K] * B[K x N] on the 64x64 tile (ty, tx); K <= KMAX.
// Column-major operands.  Four waves, each owning a 32x32 quarter computed as
// 2x2 MFMA blocks.  The MFMA computes the transposed product (B^T A^T): its
// columns are rows of C, so the 16 lanes of a lane group store 16 consecutive
// rows of one column of C (128-byte runs for FP64).
template <typename T, int KMAX>
__device__ __forceinline__ void gemm_sub_tile(T* __restrict__ C, int64_t ldc, const T* __restrict__ A,
                                              int64_t lda, const T* __restrict__ B, int64_t ldb, int M,
                                              int N, int K, int ty, int tx, T* sA, T* sB) {
  const int tid = threadIdx.x;
  const int r0 = ty * TILE, c0 = tx * TILE;
  const int Kp = (K + 3) & ~3;
  // sA[k*64 + r] = A[r0 + r, k];  sB[k*64 + c] = B[k, c0 + c]   (zero padded)
  for (int e = tid; e < Kp * TILE; e += 256) {
    const int r = e & (TILE - 1), k = e >> 6;
    const int gr = r0 + r;
    sA[e] = (gr < M && k < K) ? A[gr + (int64_t)k * lda] : T(0);
  }
  for (int e = tid; e < Kp * TILE; e += 256) {
    const int k = e % Kp, c = e / Kp;
    const int gc = c0 + c;
    sB[k * TILE + c] = (gc < N && k < K) ? B[k + (int64_t)gc * ldb] : T(0);
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int wy = w >> 1, wx = w & 1;
  typedef typename Mfma<T>::v4 v4;
  v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  for (int kk = 0; kk < Kp; kk += 4) {
    T av[2], bv[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) av[rb] = sA[(kk + lk) * TILE + wy * 32 + rb * 16 + li];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) bv[cb] = sB[(kk + lk) * TILE + wx * 32 + cb * 16 + li];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) acc[cb][rb] = Mfma<T>::mac(bv[cb], av[rb], acc[cb][rb]);
  }
  // acc[cb][rb][q]: output column c0 + wx*32 + cb*16 + row(lk, q), row r0 + wy*32 + rb*16 + li
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = r0 + wy * 32 + rb * 16 + li;
        const int gc = c0 + wx * 32 + cb * 16 + Mfma<T>::row(lk, q);
        if (gr < M && gc < N) C[gr + (int64_t)gc * ldc] -= acc[cb][rb][q];
      }
}

// C[M x N] -= A[M x K] * B[K x N] on the 64x64 tile (ty, tx), K <= KMAX, without
// LDS: each wave (32x32 quarter, 2x2 MFMA blocks) takes K in phases of S
// MFMA steps (8 for FP32, 4 for FP64) and loads the operand fragments of
// phase p + 1 straight into registers while the MFMA chain of phase p runs
// (two register buffers).  The C values are loaded after the first phase's
// operands, so that waiting for those does not wait for C; C is needed only
// at the end.  The MFMA sequence is the same for every phase length (bit-
// identical results).  Same transposed product and C layout as gemm_sub_tile.
// B_ROWS: B is stored by rows (B[k][c] at B[c + k * ldb]), so the 16 lanes of
// a lane group read 16 consecutive values of one row.
template <typename T, int KMAX, bool B_ROWS = false>
__device__ __forceinline__ void gemm_sub_tile_direct(T* __restrict__ C, int64_t ldc, const T* __restrict__ A,
                                                     int64_t lda, const T* __restrict__ B, int64_t ldb, int M, int N,
                                                     int K, int ty, int tx) {
  constexpr int SP = sizeof(T) == 8 ? 4 : 8;
  constexpr int S = KMAX / 4 < SP ? KMAX / 4 : SP;
  constexpr int NPH = KMAX / 4 / S;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wy = w >> 1, wx = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int rbase = ty * TILE + wy * 32, cbase = tx * TILE + wx * 32;
  typedef typename Mfma<T>::v4 v4;
  T av[2][S][2], bv[2][S][2];
  auto load_phase = [&](int ph, T (&a)[S][2], T (&b)[S][2]) {
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int k = 4 * (ph * S + st) + lk;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int r = rbase + rb * 16 + li;
        a[st][rb] = (r < M && k < K) ? A[r + (int64_t)k * lda] : T(0);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int c = cbase + cb * 16 + li;
        b[st][cb] = (c < N && k < K) ? (B_ROWS ? B[c + (int64_t)k * ldb] : B[k + (int64_t)c * ldb]) : T(0);
      }
    }
  };
  load_phase(0, av[0], bv[0]);
  T cv[2][2][4];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = rbase + rb * 16 + li;
        const int gc = cbase + cb * 16 + Mfma<T>::row(lk, q);
        cv[cb][rb][q] = (gr < M && gc < N) ? C[gr + (int64_t)gc * ldc] : T(0);
      }
  v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};
#pragma unroll
  for (int ph = 0; ph < NPH; ++ph) {
    if (ph > 0 && 4 * S * ph >= K) break;
    if (ph + 1 < NPH && 4 * S * (ph + 1) < K) load_phase(ph + 1, av[(ph + 1) & 1], bv[(ph + 1) & 1]);
#pragma unroll
    for (int st = 0; st < S; ++st)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          acc[cb][rb] = Mfma<T>::mac(bv[ph & 1][st][cb], av[ph & 1][st][rb], acc[cb][rb]);
  }
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = rbase + rb * 16 + li;
        const int gc = cbase + cb * 16 + Mfma<T>::row(lk, q);
        if (gr < M && gc < N) C[gr + (int64_t)gc * ldc] = cv[cb][rb][q] - acc[cb][rb][q];
      }
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_lu_panel(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                  const int* __restrict__ dim, int* __restrict__ pivb,
                                                  const int64_t* __restrict__ poff, int* __restrict__ info,
                                                  int k, int pad) {
  const int i = blockIdx.x;
  const int n = dim[i];
  if (k >= n || n - k <= panel_reg_rows<T>()) return;   // shorter panels go to k_lu_panel_rot
  const int jb = min(NB, n - k);
  const int ld = lead_dim(n, pad);
  T* A = Ab + off[i];
  int* piv = pivb + poff[i];
  __shared__ double s_val[4];
  __shared__ int s_idx[4];
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = k; j < k + jb; ++j) {
    T* colj = A + (int64_t)j * ld;
    double best = -1.0;
    int bi = n;
    for (int r = j + tid; r < n; r += 256) {
      const double v = fabs((double)colj[r]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, WAVE);
      const int oi = __shfl_xor(bi, o, WAVE);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_val[w] = best;
      s_idx[w] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = s_val[0];
      int p = s_idx[0];
      for (int q = 1; q < 4; ++q)
        if (s_val[q] > b || (s_val[q] == b && s_idx[q] < p)) {
          b = s_val[q];
          p = s_idx[q];
        }
      if (p >= n || !(b > 0.0)) {         // zero (or NaN) column: singular
        if (info[i] == 0) info[i] = j + 1;
        if (p >= n) p = j;
      }
      piv[j] = p;
      s_p = p;
    }
    __syncthreads();
    const int p = s_p;
    if (p != j) {
      for (int c = tid; c < jb; c += 256) {
        T* cc = A + (int64_t)(k + c) * ld;
        const T t = cc[j];
        cc[j] = cc[p];
        cc[p] = t;
      }
    }
    __syncthreads();
    const T pv = colj[j];
    if (pv != T(0)) {
      for (int r = j + 1 + tid; r < n; r += 256) colj[r] = colj[r] / pv;
    }
    __syncthreads();
    for (int r = j + 1 + tid; r < n; r += 256) {
      const T l = colj[r];
      for (int c = j + 1; c < k + jb; ++c) {
        T* cc = A + (int64_t)c * ld;
        cc[r] -= l * cc[j];
      }
    }
    __syncthreads();
  }
}

// ---- tall panel of a single matrix, spread over many workgroups -------------
//
// A panel A[k:n, k:k+jb) of one large matrix (more rows than one workgroup's
// registers hold) is factored one column per launch by G workgroups of TALL_T
// threads, thread t of workgroup w owning row k + TALL_T w + t.  Launch j
// (column j) reads the column's per-workgroup pivot candidates left by the
// previous launch (value, row and the candidate row's panel values), so every
// workgroup picks the same pivot (largest magnitude, ties to the lowest row),
// applies the interchange of rows j and p to the panel columns, scales column j
// and applies the rank-1 update to its own rows, and leaves the candidates of
// column j + 1 for the next launch.  Only the owners of rows j and p write
// those rows; every other workgroup reads the pivot row from the candidate
// buffer and the displaced row j from a copy the previous launch made, so no
// workgroup reads a row another one writes in the same launch.  Buffers
// alternate between two slots by column parity.
constexpr int TALL_T = 256;
constexpr int TALL_NB = 32;

template <typename T>
struct TallBufs {
  double* val;   // [2][G] candidate magnitudes
  int* idx;      // [2][G] candidate rows
  T* cand;       // [2][G][TALL_NB] candidate rows' panel values
  T* rowj;       // [2][TALL_NB] row j + 1's panel values for the next launch
};

// Candidates of column c over rows >= c held by this thread (row r, values v[0..jb)):
// workgroup argmax, then slot `slot`.  The owner of row c also stores that row.
template <typename T>
__device__ __forceinline__ void tall_candidates(const TallBufs<T>& B, int G, int slot, int c, int k, int jb, int r,
                                                bool mine, const T* v, double* s_v, int* s_i, int* s_t) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double best = -1.0;
  int bi = 0x7fffffff;
  if (mine && r >= c) {
    T vc = v[0];
#pragma unroll
    for (int q = 1; q < TALL_NB; ++q)
      if (q == c - k) vc = v[q];
    best = fabs((double)vc);
    bi = r;
  }
  int bt = tid;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, WAVE);
    const int oi = __shfl_xor(bi, o, WAVE);
    const int ot = __shfl_xor(bt, o, WAVE);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
      bt = ot;
    }
  }
  if (lane == 0) {
    s_v[w] = best;
    s_i[w] = bi;
    s_t[w] = bt;
  }
  __syncthreads();
  double b = s_v[0];
  int p = s_i[0], pt = s_t[0];
  for (int q = 1; q < TALL_T / 64; ++q)
    if (s_v[q] > b || (s_v[q] == b && s_i[q] < p)) {
      b = s_v[q];
      p = s_i[q];
      pt = s_t[q];
    }
  const int g = blockIdx.x;
  if (tid == pt && p != 0x7fffffff) {
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q)
      if (q < jb) B.cand[((size_t)slot * G + g) * TALL_NB + q] = v[q];
  }
  if (tid == 0) {
    B.val[slot * G + g] = b;
    B.idx[slot * G + g] = p;
  }
  if (mine && r == c) {
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q)
      if (q < jb) B.rowj[slot * TALL_NB + q] = v[q];
  }
}

// Candidates of the panel's first column k.
template <typename T>
__global__ __launch_bounds__(TALL_T) void k_tall_first(const T* __restrict__ A, int ld, int n, int k, int jb, int G,
                                                       TallBufs<T> B) {
  __shared__ double s_v[TALL_T / 64];
  __shared__ int s_i[TALL_T / 64], s_t[TALL_T / 64];
  const int r = k + blockIdx.x * TALL_T + threadIdx.x;
  const bool mine = r < n;
  T v[TALL_NB];
#pragma unroll
  for (int q = 0; q < TALL_NB; ++q) v[q] = (mine && q < jb) ? A[r + (int64_t)(k + q) * ld] : T(0);
  tall_candidates<T>(B, G, 0, k, k, jb, r, mine, v, s_v, s_i, s_t);
}

// Column j of the panel [k, k + jb): pivot, interchange, scaling, rank-1 update,
// candidates of column j + 1.
template <typename T>
__global__ __launch_bounds__(TALL_T) void k_tall_step(T* __restrict__ A, int ld, int n, int k, int jb, int j, int G,
                                                      TallBufs<T> B, int* __restrict__ piv, int* __restrict__ info) {
  __shared__ double s_v[TALL_T / 64];
  __shared__ int s_i[TALL_T / 64], s_t[TALL_T / 64];
  __shared__ T s_prow[TALL_NB];
  const int slot = (j - k) & 1;
  // the pivot: every workgroup reduces the same candidates in the same order
  double bv = B.val[slot * G];
  int p = B.idx[slot * G], gw = 0;
  for (int g = 1; g < G; ++g) {
    const double v = B.val[slot * G + g];
    const int i = B.idx[slot * G + g];
    if (v > bv || (v == bv && i < p)) {
      bv = v;
      p = i;
      gw = g;
    }
  }
  const bool singular = !(bv > 0.0) || p >= n;
  if (singular) {
    p = j;
  }
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) {
    piv[j] = p;
    if (singular && info[0] == 0) info[0] = j + 1;
  }
  // the pivot row's panel values (row j's own values when the column is singular)
  for (int q = tid; q < jb; q += TALL_T)
    s_prow[q] = singular ? B.rowj[slot * TALL_NB + q] : B.cand[((size_t)slot * G + gw) * TALL_NB + q];
  __syncthreads();
  const int r = k + blockIdx.x * TALL_T + tid;
  const bool mine = r < n;
  T v[TALL_NB];
  if (mine && r == j) {
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q) v[q] = q < jb ? s_prow[q] : T(0);
  } else if (mine && r == p) {           // p != j: receives row j
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q) v[q] = q < jb ? B.rowj[slot * TALL_NB + q] : T(0);
  } else {
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q) v[q] = (mine && q < jb && r > j) ? A[r + (int64_t)(k + q) * ld] : T(0);
  }
  const int cj = j - k;
  if (mine && r > j) {
    const T pv = s_prow[cj];
    const T l = (pv != T(0)) ? v[cj] / pv : v[cj];
    v[cj] = l;
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q)
      if (q > cj && q < jb) v[q] -= l * s_prow[q];
  }
  // stores: row j (the pivot row), row p (old row j, updated), and every other row below j
  if (mine && (r > j || r == j)) {
    if (r == j || r == p) {
      for (int q = 0; q < jb; ++q) A[r + (int64_t)(k + q) * ld] = v[q];
    } else {
      for (int q = cj; q < jb; ++q) A[r + (int64_t)(k + q) * ld] = v[q];
    }
  }
  if (j + 1 < k + jb) tall_candidates<T>(B, G, slot ^ 1, j + 1, k, jb, r, mine && r > j, v, s_v, s_i, s_t);
}

// The whole panel [k, k + jb) in one cooperative launch: the same column steps
// as k_tall_first + k_tall_step (same candidates, pivot choice and arithmetic,
// hence the same factors), with every thread's row kept in registers across
// the panel's columns and a grid barrier where the per-column launches had a
// kernel boundary.  The panel is read once and written once; one launch per
// panel instead of jb + 1, which matters most when other streams keep every
// CU busy and each launch waits for free slots.
template <typename T>
__global__ __launch_bounds__(TALL_T) void k_tall_panel_coop(T* __restrict__ A, int ld, int n, int k, int jb, int G,
                                                            TallBufs<T> B, int* __restrict__ piv,
                                                            int* __restrict__ info) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  __shared__ double s_v[TALL_T / 64];
  __shared__ int s_i[TALL_T / 64], s_t[TALL_T / 64];
  __shared__ T s_prow[TALL_NB];
  const int tid = threadIdx.x;
  const int r = k + blockIdx.x * TALL_T + tid;
  const bool mine = r < n;
  T v[TALL_NB];
#pragma unroll
  for (int q = 0; q < TALL_NB; ++q) v[q] = (mine && q < jb) ? A[r + (int64_t)(k + q) * ld] : T(0);
  tall_candidates<T>(B, G, 0, k, k, jb, r, mine, v, s_v, s_i, s_t);
  for (int j = k; j < k + jb; ++j) {
    grid.sync();                       // every workgroup's candidates of column j are out
    const int slot = (j - k) & 1;
    double bv = B.val[slot * G];
    int p = B.idx[slot * G], gw = 0;
    for (int g = 1; g < G; ++g) {
      const double cv = B.val[slot * G + g];
      const int ci = B.idx[slot * G + g];
      if (cv > bv || (cv == bv && ci < p)) {
        bv = cv;
        p = ci;
        gw = g;
      }
    }
    const bool singular = !(bv > 0.0) || p >= n;
    if (singular) p = j;
    if (blockIdx.x == 0 && tid == 0) {
      piv[j] = p;
      if (singular && info[0] == 0) info[0] = j + 1;
    }
    for (int q = tid; q < jb; q += TALL_T)
      s_prow[q] = singular ? B.rowj[slot * TALL_NB + q] : B.cand[((size_t)slot * G + gw) * TALL_NB + q];
    __syncthreads();
    if (mine && r == j) {
#pragma unroll
      for (int q = 0; q < TALL_NB; ++q) v[q] = q < jb ? s_prow[q] : T(0);
    } else if (mine && r == p) {       // p != j: receives row j
#pragma unroll
      for (int q = 0; q < TALL_NB; ++q) v[q] = q < jb ? B.rowj[slot * TALL_NB + q] : T(0);
    }
    const int cj = j - k;
    if (mine && r > j) {
      T vc = v[0];
#pragma unroll
      for (int q = 1; q < TALL_NB; ++q)
        if (q == cj) vc = v[q];
      const T pv = s_prow[cj];
      const T l = (pv != T(0)) ? vc / pv : vc;
#pragma unroll
      for (int q = 0; q < TALL_NB; ++q) {
        if (q == cj) v[q] = l;
        if (q > cj && q < jb) v[q] -= l * s_prow[q];
      }
    }
    if (j + 1 < k + jb) tall_candidates<T>(B, G, slot ^ 1, j + 1, k, jb, r, mine && r > j, v, s_v, s_i, s_t);
  }
  if (mine) {
#pragma unroll
    for (int q = 0; q < TALL_NB; ++q)
      if (q < jb) A[r + (int64_t)(k + q) * ld] = v[q];
  }
}

// (ov, ol) beats (val, lab): larger value, equal values to the smaller label.
// Evaluated without short-circuit so it compiles to compares and selects.
__device__ __forceinline__ bool argmax_beats(double ov, int ol, double val, int lab) {
  return (ov > val) | ((ov == val) & (ol < lab));
}

// One DPP step of the pivot search: combine (val, lab) with the lane selected
// by CTRL (a permutation inside each row of 16 lanes).
template <int CTRL>
__device__ __forceinline__ void argmax_dpp_step(double& val, int& lab) {
  const long long bits = __builtin_bit_cast(long long, val);
  const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xf, 0xf, false);
  const int ol = __builtin_amdgcn_mov_dpp(lab, CTRL, 0xf, 0xf, false);
  const double ov = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
  const bool t = argmax_beats(ov, ol, val, lab);
  val = t ? ov : val;
  lab = t ? ol : lab;
}

// Wave-wide argmax of (val, lab); every lane receives the winner.  Butterflies
// inside each 16-lane row (quad_perm [1,0,3,2], [2,3,0,1], half mirror,
// mirror), then the four row winners are combined from lanes 0, 16, 32, 48.
__device__ __forceinline__ void wave_argmax(double& val, int& lab) {
  argmax_dpp_step<0xB1>(val, lab);
  argmax_dpp_step<0x4E>(val, lab);
  argmax_dpp_step<0x141>(val, lab);
  argmax_dpp_step<0x140>(val, lab);
  double rv[4];
  int rl[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    rv[r] = lane_value(val, 16 * r);
    rl[r] = lane_value(lab, 16 * r);
  }
  double b = rv[0];
  int l = rl[0];
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const bool t = argmax_beats(rv[r], rl[r], b, l);
    b = t ? rv[r] : b;
    l = t ? rl[r] : l;
  }
  val = b;
  lab = l;
}

constexpr int NO_ROW = 0x7fffffff;

// Register-resident panel factorization of A[k:n, k:k+NB] for panels of at most
// NT * R rows, one workgroup per matrix.  Thread t holds panel rows t + NT q
// (q < R).  Rows never move while the panel is factored: each carries a label,
// its position in the interchanged order, and an interchange swaps two labels;
// at the end every row is stored at its label.
//
// Columns are processed in chunks of 8 with the 8 steps of a chunk unrolled
// (static register indices); the loop over chunks is not unrolled, so the
// code stays small.  After a chunk the registers of each row rotate by 8:
// the current chunk is always registers 0..7, the columns still to factor
// follow, and finished chunks collect at the top (after NB / 8 chunks the
// original order is back).  Blocks of 8 finished columns are skipped by the
// rank-1 update with a wavefront-uniform branch.
//
// Per column: every thread proposes its best candidate (largest |a| among rows
// at or below the diagonal, ties to the smallest label), waves reduce with DPP,
// each wave's winner writes value, label and its row to a double-buffered LDS
// slot, one barrier, and every thread picks the winning wave and applies the
// rank-1 update from that slot.  Nothing is stored to global memory inside the
// column loop (pivot indices and the singularity flag are written after it),
// so the barriers never wait on global stores.
template <typename T, int NB, int NT, int R>
__global__ __launch_bounds__(NT, (sizeof(T) == 8 && NT == 256 && R == 3) ? 2 : 1) void k_lu_panel_rot(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                     const int* __restrict__ dim, int* __restrict__ pivb,
                                                     const int64_t* __restrict__ poff, int* __restrict__ info,
                                                     int k, int pad, const int* __restrict__ list = nullptr,
                                                     int first = 0) {
  static_assert(NB % 8 == 0, "panel width must be a multiple of 8");
  constexpr int NW = NT / 64;
  constexpr int CH = 8;
  // list: the matrices of one size class (a range of the batch sorted by decreasing order)
  const int i = list ? list[first + blockIdx.x] : blockIdx.x;
  const int n = dim[i];
  const int m = n - k;
  if (m <= 0 || m > NT * R) return;         // taller panels go to k_lu_panel
  const int jb = min(NB, m);
  const int ld = lead_dim(n, pad);
  T* A = Ab + off[i] + k + (int64_t)k * ld;  // panel origin
  int* piv = pivb + poff[i] + k;
  __shared__ double s_val[2][NW];
  __shared__ int s_lab[2][NW];
  __shared__ T s_row[2 * NW * NB];          // [buffer][wave][column]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  T v[R][NB];
  int lab[R];
  int piv_r = 0;                            // lane j of wave 0 keeps pivot j
  int first_zero = 0;                       // 1 + first column without a nonzero pivot
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + NT * q;
    lab[q] = r < m ? r : NO_ROW;
#pragma unroll
    for (int c = 0; c < NB; ++c) v[q][c] = (r < m && c < jb) ? A[r + (int64_t)c * ld] : T(0);
  }
#pragma clang loop unroll(disable)
  for (int g = 0; g < NB / CH; ++g) {
    const int live = NB / CH - g;           // 8-column blocks not yet finished (block 0 = this chunk)
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      const int j = CH * g + jj;
      if (j >= jb) break;
      const int buf = j & 1;
      double best = -1.0;
      int bl = NO_ROW, bq = -1;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const double a = fabs((double)v[q][jj]);
        const bool t = (lab[q] >= j) & (lab[q] != NO_ROW) & argmax_beats(a, lab[q], best, bl);
        best = t ? a : best;
        bl = t ? lab[q] : bl;
        bq = t ? q : bq;
      }
      double wb = best;
      int wl = bl;
      wave_argmax(wb, wl);
      if (lane == 0) {
        s_val[buf][w] = wb;
        s_lab[buf][w] = wl;
      }
      if (wl != NO_ROW && bl == wl) {        // this wave's winner publishes its row
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (bq == q) {
#pragma unroll
            for (int c = jj; c < NB; ++c) s_row[(buf * NW + w) * NB + c] = v[q][c];
          }
      }
      __syncthreads();
      double wv[NW];
      int wlab[NW];
#pragma unroll
      for (int x = 0; x < NW; ++x) {
        wv[x] = s_val[buf][x];
        wlab[x] = s_lab[buf][x];
      }
      double b = wv[0];
      int p = wlab[0], pw = 0;
#pragma unroll
      for (int x = 1; x < NW; ++x) {
        const bool t = argmax_beats(wv[x], wlab[x], b, p);
        b = t ? wv[x] : b;
        p = t ? wlab[x] : p;
        pw = t ? x : pw;
      }
      const bool have = (p != NO_ROW);       // false only when every candidate is NaN
      if (tid == j) piv_r = k + (have ? p : j);
      if ((!have || !(b > 0.0)) && first_zero == 0) first_zero = j + 1;
      if (!have) continue;
#pragma unroll
      for (int q = 0; q < R; ++q) lab[q] = (lab[q] == j) ? p : (lab[q] == p ? j : lab[q]);
      const int src = (buf * NW + pw) * NB;
      const T pv = s_row[src + jj];
      T l[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const bool below = lab[q] > j && lab[q] != NO_ROW;
        l[q] = below ? ((pv != T(0)) ? v[q][jj] / pv : v[q][jj]) : T(0);
        v[q][jj] = below ? l[q] : v[q][jj];
      }
#pragma unroll
      for (int c = jj + 1; c < CH; ++c) {
        const T uc = s_row[src + c];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q][c] -= l[q] * uc;
      }
#pragma unroll
      for (int bk = 1; bk < NB / CH; ++bk)
        if (bk < live) {
#pragma unroll
          for (int c = CH * bk; c < CH * bk + CH; ++c) {
            const T uc = s_row[src + c];
#pragma unroll
            for (int q = 0; q < R; ++q) v[q][c] -= l[q] * uc;
          }
        }
    }
    // rotate each row by one chunk
#pragma unroll
    for (int q = 0; q < R; ++q) {
      T t[CH];
#pragma unroll
      for (int x = 0; x < CH; ++x) t[x] = v[q][x];
#pragma unroll
      for (int c = 0; c < NB - CH; ++c) v[q][c] = v[q][c + CH];
#pragma unroll
      for (int x = 0; x < CH; ++x) v[q][NB - CH + x] = t[x];
    }
  }
  if (tid < jb) piv[tid] = piv_r;
  if (tid == 0 && first_zero && info[i] == 0) info[i] = k + first_zero;
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (lab[q] != NO_ROW) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < jb) A[lab[q] + (int64_t)c * ld] = v[q][c];
    }
}

// ---- two-level blocking: outer width 2 * NB, two NB-wide sub-panels ----------

// Sub-panel 1 of outer step k is factored; bring columns [k+NB, k+2NB) up to
// date: its interchanges, then U = L11^{-1} A on rows [k, k+NB).
template <typename T, int NB>
__global__ __launch_bounds__(64) void k_lu_inner_swap_trsm(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                           const int* __restrict__ dim, const int* __restrict__ pivb,
                                                           const int64_t* __restrict__ poff, int k, int pad) {
  const int i = blockIdx.x;
  const int n = dim[i];
  if (k + NB >= n) return;                  // no second sub-panel
  const int ld = lead_dim(n, pad);
  T* A = Ab + off[i];
  const int* piv = pivb + poff[i];
  __shared__ T L11[NB * NB];
  for (int t = threadIdx.x; t < NB * NB; t += 64) {
    const int r = t % NB, c = t / NB;
    L11[t] = A[(k + r) + (int64_t)(k + c) * ld];
  }
  __syncthreads();
  const int c = k + NB + (int)threadIdx.x;
  if (threadIdx.x >= NB || c >= n) return;
  T* col = A + (int64_t)c * ld;
  for (int j = k; j < k + NB; ++j) {
    const int p = piv[j];
    if (p != j) {
      const T t = col[j];
      col[j] = col[p];
      col[p] = t;
    }
  }
  T x[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) x[r] = col[k + r];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = j + 1; r < NB; ++r) x[r] -= L11[r + j * NB] * x[j];
#pragma unroll
  for (int r = 0; r < NB; ++r) col[k + r] = x[r];
}

// After both sub-panels of outer step k: interchanges on the columns left of
// sub-panel 2 (all pivots of the step left of k; sub-panel 2's pivots on
// sub-panel 1).
template <typename T, int NB>
__global__ __launch_bounds__(64) void k_lu_outer_swap_left(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                           const int* __restrict__ dim, const int* __restrict__ pivb,
                                                           const int64_t* __restrict__ poff, int k, int pad) {
  const int i = blockIdx.x;
  const int n = dim[i];
  if (k >= n) return;
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= k + NB || c >= n) return;
  const int kw = min(2 * NB, n - k);
  T* col = Ab + off[i] + (int64_t)c * lead_dim(n, pad);
  const int* piv = pivb + poff[i];
  for (int j = (c < k ? k : k + NB); j < k + kw; ++j) {
    const int p = piv[j];
    if (p != j) {
      const T t = col[j];
      col[j] = col[p];
      col[p] = t;
    }
  }
}

// Interchanges piv[j0, j0 + nj) applied in order to columns [c0, c0 + nc).
template <typename T>
__global__ __launch_bounds__(64) void k_lu_swap_cols(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                     const int* __restrict__ dim, const int* __restrict__ pivb,
                                                     const int64_t* __restrict__ poff, int j0, int nj, int c0, int nc,
                                                     int pad) {
  const int i = blockIdx.x;
  const int n = dim[i];
  const int c = c0 + blockIdx.y * 64 + (int)threadIdx.x;
  if (c >= c0 + nc || c >= n) return;
  T* col = Ab + off[i] + (int64_t)c * lead_dim(n, pad);
  const int* piv = pivb + poff[i];
  const int j1 = min(j0 + nj, n);
  for (int j = j0; j < j1; ++j) {
    const int p = piv[j];
    if (p != j) {
      const T t = col[j];
      col[j] = col[p];
      col[p] = t;
    }
  }
}

// Columns right of outer step k: all of its interchanges, then
// U12 = L11^{-1} A12 with the 2NB x 2NB unit lower L11.  One thread per
// column, TRSM_COLS columns per workgroup; L11 and the step's pivots are staged
// in LDS once per workgroup.
constexpr int TRSM_COLS = 128;
template <typename T, int NB>
__global__ __launch_bounds__(TRSM_COLS) void k_lu_outer_swap_trsm(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                                  const int* __restrict__ dim,
                                                                  const int* __restrict__ pivb,
                                                                  const int64_t* __restrict__ poff, int k, int pad,
                                                                  T* __restrict__ ut, int swap, int ut_rows,
                                                                  int ut_row0, int ut_k0) {
  constexpr int KW = 2 * NB;
  const int i = blockIdx.x;
  const int n = dim[i];
  const int cfirst = k + KW + blockIdx.y * TRSM_COLS;
  if (cfirst >= n) return;                  // no trailing columns in this block
  const int ld = lead_dim(n, pad);
  T* A = Ab + off[i];
  const int* piv = pivb + poff[i];
  __shared__ T L11[KW * KW];
  __shared__ int sp[KW];
  for (int t = threadIdx.x; t < KW * KW; t += TRSM_COLS) {
    const int r = t % KW, c = t / KW;
    L11[t] = A[(k + r) + (int64_t)(k + c) * ld];
  }
  if (threadIdx.x < KW) sp[threadIdx.x] = piv[k + threadIdx.x];
  __syncthreads();
  const int c = cfirst + (int)threadIdx.x;
  if (c >= n) return;
  T* col = A + (int64_t)c * ld;
  if (swap) {
    for (int j = 0; j < KW; ++j) {
      const int p = sp[j];
      if (p != k + j) {
        const T t = col[k + j];
        col[k + j] = col[p];
        col[p] = t;
      }
    }
  }
  // padded columns (pad > 1: 128-byte aligned) move their 64 values in 16-byte pieces
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  T x[KW];
  if (pad > 1) {
    const vec* src = reinterpret_cast<const vec*>(col + k);
#pragma unroll
    for (int r = 0; r < KW / V; ++r) {
      const vec v = src[r];
#pragma unroll
      for (int e = 0; e < V; ++e) x[V * r + e] = v[e];
    }
  } else {
#pragma unroll
    for (int r = 0; r < KW; ++r) x[r] = col[k + r];
  }
#pragma unroll
  for (int j = 0; j < KW; ++j)
#pragma unroll
    for (int r = j + 1; r < KW; ++r) x[r] -= L11[r + j * KW] * x[j];
  if (pad > 1) {
    vec* dst = reinterpret_cast<vec*>(col + k);
#pragma unroll
    for (int r = 0; r < KW / V; ++r) {
      vec v;
#pragma unroll
      for (int e = 0; e < V; ++e) v[e] = x[V * r + e];
      dst[r] = v;
    }
  } else {
#pragma unroll
    for (int r = 0; r < KW; ++r) col[k + r] = x[r];
  }
  if (ut) {   // U12 by rows into the scratch: ut_rows rows of length n - ut_k0 - KW per matrix
    const int M = n - ut_k0 - KW;
    T* u = ut + (int64_t)ut_rows * poff[i] + (int64_t)ut_row0 * M + (c - ut_k0 - KW);
#pragma unroll
    for (int r = 0; r < KW; ++r) u[(int64_t)r * M] = x[r];
  }
}

// A[r0:n, c0:c1) -= A[r0:n, k:k+kw) * A[k:k+kw, c0:c1), r0 = k + kw (64x64 MFMA tiles).
// inner = 1: kw = NB, c0 = k+NB, c1 = k+2NB (sub-panel 2 before its factorization);
// inner = 0: kw = 2NB, c0 = k+2NB, c1 = n (trailing matrix).
// ut (outer steps only, may be null): the step's U12 by rows at 64 * poff[i].
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_lu_update(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                   const int* __restrict__ dim, int k, int inner, int tiles_m,
                                                   int tiles_n, const int64_t* __restrict__ tab, int count, int pad,
                                                   const T* __restrict__ ut, const int64_t* __restrict__ poff) {
  const int w = (int)xcd_remap(blockIdx.x, gridDim.x);
  int i, tl;
  if (tab) {                                // compact grid: tab[i] = first tile of matrix i
    i = segment_of(tab, count, w);
    tl = w - (int)tab[i];
  } else {
    const int tiles = tiles_m * tiles_n;
    i = w / tiles;
    tl = w - i * tiles;
  }
  const int n = dim[i];
  const int kw = inner ? NB : 2 * NB;
  if (k + kw >= n) return;
  const int r0 = k + kw;
  const int c0 = inner ? k + NB : k + 2 * NB;
  const int c1 = inner ? min(n, k + 2 * NB) : n;
  const int M = n - r0, N = c1 - c0;
  const int tm = tab ? (M + TILE - 1) / TILE : tiles_m;
  const int ty = tl % tm, tx = tl / tm;
  if (ty * TILE >= M || tx * TILE >= N) return;
  const int ld = lead_dim(n, pad);
  T* A = Ab + off[i];
  if (!inner && ut)
    gemm_sub_tile_direct<T, 2 * NB, true>(A + r0 + (int64_t)c0 * ld, ld, A + r0 + (int64_t)k * ld, ld,
                                          ut + 64 * poff[i], N, M, N, kw, ty, tx);
  else
    gemm_sub_tile_direct<T, 2 * NB>(A + r0 + (int64_t)c0 * ld, ld, A + r0 + (int64_t)k * ld, ld,
                                    A + k + (int64_t)c0 * ld, ld, M, N, kw, ty, tx);
}

// Zero tiles of the operands of the rank-4NB trailing update of the pair at k0 (wide steps):
// bit t of masks[2 i] is set when rows [r0 + 64 t, r0 + 64 t + 64) of columns [k0, k0 + 4NB) of
// matrix i (L21, r0 = k0 + 4NB) hold a nonzero, bit t of masks[2 i + 1] when columns
// [c0 + 64 t, ...) of the 4NB rows of U12 (row-major scratch, c0 = k0 + 4NB) do.  Tiles from the
// 65th on are not tracked (k_lu_update_ut treats them as nonzero).  One workgroup per matrix.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_step_masks(const T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                       const int* __restrict__ dim, int k0, int pad,
                                                       const T* __restrict__ ut, const int64_t* __restrict__ poff,
                                                       int ut_rows, unsigned long long* __restrict__ masks) {
  __shared__ unsigned long long lm, um;
  constexpr int KW = 4 * LU_NB;
  const int i = blockIdx.x;
  const int n = dim[i];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) lm = um = 0ull;
  __syncthreads();
  const int r0 = k0 + KW;
  if (r0 < n) {
    const int ld = lead_dim(n, pad);
    const T* A = Ab + off[i];
    const int tl = min(64, (n - r0 + TILE - 1) / TILE);
    for (int t = wid; t < tl; t += 4) {          // L21: lane = row, over the 4NB columns
      const int row = r0 + t * TILE + lane;
      bool nz = false;
      if (row < n) {
        int64_t o = row + (int64_t)k0 * ld;
#pragma unroll 16
        for (int c = 0; c < KW; ++c) {
          nz |= A[o] != T(0);
          o += ld;
        }
      }
      if (__any(nz) && lane == 0) atomicOr(&lm, 1ull << t);
    }
    const int urow = n - k0 - 2 * LU_NB;        // U12 rows: columns k0 + 2NB ... n - 1
    const T* U = ut + (int64_t)ut_rows * poff[i] + (r0 - k0 - 2 * LU_NB);
    for (int t = wid; t < tl; t += 4) {          // U12: lane = column, over the 4NB rows
      const int c = t * TILE + lane;
      bool nz = false;
      if (r0 + c < n) {
        const T* u = U + c;
#pragma unroll 16
        for (int k = 0; k < KW; ++k) nz |= u[(int64_t)k * urow] != T(0);
      }
      if (__any(nz) && lane == 0) atomicOr(&um, 1ull << t);
    }
  }
  __syncthreads();
  if (tid == 0) {
    masks[2 * i] = lm;
    masks[2 * i + 1] = um;
  }
}

// Updates of the paired-step factorization (lu_batched, wide): with k0 the
// first column of the pair,
//   A[r0 : r0 + M, c0 : c1) -= A[r0 : r0 + M, k0 : k0 + kw) * U[0 : kw, c0 : c1)
// r0 = k0 + r0_rel, M = min(n - r0, m_cap), c0 = k0 + c0_rel, c1 = k0 + c1_rel (n if c1_rel < 0).
// U's rows come from the row-major scratch (rows of length n - k0 - 64 starting
// at column k0 + 64, matrix i at ut_rows * poff[i]).
// masks (may be null): words 2i and 2i + 1 from k_lu_step_masks; a C tile whose 64 rows of the A
// operand or 64 columns of U are all zero is left as it is (its product is an exact zero).
template <typename T, int KMAX>
__global__ __launch_bounds__(256) void k_lu_update_ut(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                      const int* __restrict__ dim, int k0, int r0_rel, int m_cap,
                                                      int c0_rel, int c1_rel, int kw, int tiles_m, int tiles_n,
                                                      const int64_t* __restrict__ tab, int count, int pad,
                                                      const T* __restrict__ ut, const int64_t* __restrict__ poff,
                                                      int ut_rows, const unsigned long long* __restrict__ masks) {
  const int w = (int)xcd_remap(blockIdx.x, gridDim.x);
  int i, tl;
  if (tab) {
    i = segment_of(tab, count, w);
    tl = w - (int)tab[i];
  } else {
    const int tiles = tiles_m * tiles_n;
    i = w / tiles;
    tl = w - i * tiles;
  }
  const int n = dim[i];
  const int r0 = k0 + r0_rel;
  if (r0 >= n) return;
  const int M = min(n - r0, m_cap);
  const int c0 = k0 + c0_rel;
  const int c1 = c1_rel < 0 ? n : min(n, k0 + c1_rel);
  if (c0 >= c1) return;
  const int N = c1 - c0;
  const int tm = tab ? (M + TILE - 1) / TILE : tiles_m;
  const int ty = tl % tm, tx = tl / tm;
  if (ty * TILE >= M || tx * TILE >= N) return;
  if (masks) {
    const unsigned long long lm = masks[2 * i], um = masks[2 * i + 1];
    if ((ty < 64 && !((lm >> ty) & 1ull)) || (tx < 64 && !((um >> tx) & 1ull))) return;
  }
  const int ld = lead_dim(n, pad);
  T* A = Ab + off[i];
  const int urow = n - k0 - 2 * LU_NB;
  const T* U = ut + (int64_t)ut_rows * poff[i] + (c0 - k0 - 2 * LU_NB);
  gemm_sub_tile_direct<T, KMAX, true>(A + r0 + (int64_t)c0 * ld, ld, A + r0 + (int64_t)k0 * ld, ld, U, urow, M, N, kw,
                                      ty, tx);
}

// mode 0: LU trailing update; 1: forward-solve update of X; 2: backward-solve update of X.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_gemm_update(T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                     const int* __restrict__ dim, T* __restrict__ Xb,
                                                     const int64_t* __restrict__ xoff, const int* __restrict__ nrhs,
                                                     int k, int mode, int tiles_n) {
  // logical index = tile + tiles_n^2 * matrix; tiles are (ty, tx) with ty fastest
  const int tiles = tiles_n * tiles_n;
  const int w = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = w / tiles;
  const int tl = w - i * tiles;
  const int n = dim[i];
  if (k >= n) return;
  const int jb = min(NB, n - k);
  const int ty = tl % tiles_n;
  const int tx = tl / tiles_n;
  T* A = Ab + off[i];
  int M, N;
  T* C;
  const T *Ap, *Bp;
  int64_t ldc, ldb;
  if (mode == 0) {
    M = N = n - k - jb;
    C = A + (k + jb) + (int64_t)(k + jb) * n;
    Ap = A + (k + jb) + (int64_t)k * n;
    Bp = A + k + (int64_t)(k + jb) * n;
    ldc = ldb = n;
  } else {
    T* X = Xb + xoff[i];
    N = nrhs[i];
    ldc = ldb = n;
    if (mode == 1) {
      M = n - k - jb;
      C = X + (k + jb);
      Ap = A + (k + jb) + (int64_t)k * n;
      Bp = X + k;
    } else {
      M = k;
      C = X;
      Ap = A + (int64_t)k * n;
      Bp = X + k;
    }
  }
  if (ty * TILE >= M || tx * TILE >= N) return;
  gemm_sub_tile_direct<T, NB>(C, ldc, Ap, n, Bp, ldb, M, N, jb, ty, tx);
}

// Row interchanges of the whole factorization applied to each right-hand side.
template <typename T>
__global__ void k_getrs_swap(const int* __restrict__ dim, const int* __restrict__ pivb,
                             const int64_t* __restrict__ poff, T* __restrict__ Xb,
                             const int64_t* __restrict__ xoff, const int* __restrict__ nrhs) {
  const int i = blockIdx.x;
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= nrhs[i]) return;
  const int n = dim[i];
  const int* piv = pivb + poff[i];
  T* x = Xb + xoff[i] + (int64_t)c * n;
  for (int j = 0; j < n; ++j) {
    const int p = piv[j];
    if (p != j) {
      const T t = x[j];
      x[j] = x[p];
      x[p] = t;
    }
  }
}

// Diagonal block solve of the forward (unit L) or backward (U) sweep for rows k..k+jb.
template <typename T, int NB>
__global__ __launch_bounds__(64) void k_getrs_diag(const T* __restrict__ Ab, const int64_t* __restrict__ off,
                                                   const int* __restrict__ dim, T* __restrict__ Xb,
                                                   const int64_t* __restrict__ xoff, const int* __restrict__ nrhs,
                                                   int k, int upper) {
  const int i = blockIdx.x;
  const int n = dim[i];
  if (k >= n) return;
  const int jb = min(NB, n - k);
  const T* A = Ab + off[i];
  __shared__ T D[NB * NB];
  for (int t = threadIdx.x; t < jb * jb; t += 64) {
    const int r = t % jb, c = t / jb;
    D[t] = A[(k + r) + (int64_t)(k + c) * n];
  }
  __syncthreads();
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= nrhs[i]) return;
  T* col = Xb + xoff[i] + (int64_t)c * n + k;
  T x[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) x[r] = (r < jb) ? col[r] : T(0);
  if (!upper) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < jb) {
#pragma unroll
        for (int r = j + 1; r < NB; ++r)
          if (r < jb) x[r] -= D[r + j * jb] * x[j];
      }
  } else {
#pragma unroll
    for (int j = NB - 1; j >= 0; --j)
      if (j < jb) {
        x[j] = x[j] / D[j + j * jb];
#pragma unroll
        for (int r = 0; r < NB; ++r)
          if (r < j) x[r] -= D[r + j * jb] * x[j];
      }
  }
#pragma unroll
  for (int r = 0; r < NB; ++r)
    if (r < jb) col[r] = x[r];
}

// ---- explicit inverse of one large LU-factored matrix --------------------
//
// X = A^{-1} from P A = L U (X starts as P I): forward sweep with L, backward
// with U, both in 128-row blocks of four 32-row diagonal solves; the rows past
// a block are updated once per block with inner dimension 128 (a quarter of the
// passes over X of a 32-row blocking).  In the forward sweep, column c of P I
// is zero above the row q with perm[q] = c, and stays so: a 64-column tile of X
// whose columns all start below the block is skipped (lo[tile] = first row of
// the tile's columns that can be nonzero).

// X[r0 : r0 + M, 0 : n) -= A[r0 : r0 + M, kc : kc + kw) X[kc : kc + kw, 0 : n) (leading dimension n).
template <typename T, int KMAX>
__global__ __launch_bounds__(256) void k_inv_update(const T* __restrict__ A, T* __restrict__ X, int n, int r0, int M,
                                                    int kc, int kw, int tiles_m, const int* __restrict__ lo) {
  const int w = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int ty = w % tiles_m, tx = w / tiles_m;
  if (lo && lo[tx] >= kc + kw) return;
  gemm_sub_tile_direct<T, KMAX>(X + r0, n, A + r0 + (int64_t)kc * n, n, X + kc, n, M, n, kw, ty, tx);
}

// lo[t] = min over the columns c of tile t of the position q with perm[q] = c.
__global__ void k_inv_first_rows(const int* __restrict__ perm, int n, int* __restrict__ pinv, int* __restrict__ lo,
                                 int phase) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (phase == 0) {
    if (t < n) pinv[perm[t]] = t;
  } else {
    if (t * TILE >= n) return;
    int m = n;
    for (int c = t * TILE; c < min(n, (t + 1) * TILE); ++c) m = min(m, pinv[c]);
    lo[t] = m;
  }
}

// perm[r] = original row at position r after the interchanges piv[0..n) of
// matrix blockIdx.x, applied in order.  The permutation lives in LDS while one
// thread applies the interchanges (orders up to PERM_LDS; longer ones in global
// memory).
constexpr int PERM_LDS = 4096;
__global__ __launch_bounds__(256) void k_build_perm(const int* __restrict__ dim, const int* __restrict__ pivb,
                                                    const int64_t* __restrict__ poff, int* __restrict__ perm) {
  __shared__ int sp[PERM_LDS];
  const int i = blockIdx.x;
  const int n = dim[i];
  const int* piv = pivb + poff[i];
  int* p = perm + poff[i];
  if (n > PERM_LDS) {
    if (threadIdx.x == 0) {
      for (int a = 0; a < n; ++a) p[a] = a;
      for (int j = 0; j < n; ++j) {
        const int q = piv[j];
        if (q != j) {
          const int t = p[j];
          p[j] = p[q];
          p[q] = t;
        }
      }
    }
    return;
  }
  for (int a = threadIdx.x; a < n; a += blockDim.x) sp[a] = a;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < n; ++j) {
      const int q = piv[j];
      if (q != j) {
        const int t = sp[j];
        sp[j] = sp[q];
        sp[q] = t;
      }
    }
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += blockDim.x) p[a] = sp[a];
}

// Inverse of one LU-factored matrix (P A = L U) with the solution resident in
// registers: workgroup b owns right-hand-side columns [NC b, NC b + NC) of
// P I, thread t holds rows t + 512 q (q < R) of them through the forward sweep
// with unit L and the backward sweep with U, in 32-row diagonal blocks.  Per
// block the owners put its rows into LDS, the 32 x 32 triangle is solved with
// one 32-lane group per column (lane i holds row i; step j broadcasts lane j
// by shuffle), and every thread updates its own rows below (forward) or above
// (backward) with VALU FMAs, all loads of a row issued first.  The result is stored transposed:
// out[c + r n] = (A^{-1})[r][c], i.e. A^{-1} by rows.
template <typename T, int R, int NC>
__global__ __launch_bounds__(512) void k_inverse_resident(const T* __restrict__ A, const int* __restrict__ perm,
                                                          T* __restrict__ out, int n) {
  constexpr int NT = 512, KB = 32;
  __shared__ T sX[KB][NC];
  __shared__ T sD[KB][KB + 1];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * NC;
  T x[R][NC];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + NT * q;
    const int pr = (r < n) ? perm[r] : -1;
#pragma unroll
    for (int c = 0; c < NC; ++c) x[q][c] = (pr == c0 + c) ? T(1) : T(0);
  }
  // forward: L Y = P I
  for (int kb = 0; kb < n; kb += KB) {
    const int kw = min(KB, n - kb);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r >= kb && r < kb + kw)
#pragma unroll
        for (int c = 0; c < NC; ++c) sX[r - kb][c] = x[q][c];
    }
    for (int e = tid; e < kw * kw; e += NT) {
      const int i = e % kw, j = e / kw;
      sD[i][j] = A[(kb + i) + (int64_t)(kb + j) * n];
    }
    __syncthreads();
    if (tid < 32 * NC) {                    // lane group of 32: row i of column c
      const int i = tid & 31, c = tid >> 5, base = tid & 32;
      T y = (i < kw) ? sX[i][c] : T(0);
      for (int j = 0; j < kw; ++j) {
        const T yj = __shfl(y, base + j, WAVE);
        if (i > j) y -= sD[i][j] * yj;
      }
      if (i < kw) sX[i][c] = y;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r >= kb && r < kb + kw) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[q][c] = sX[r - kb][c];
      } else if (r >= kb + kw && r < n) {
        T lv[KB];                           // all loads of the row issued before the FMAs
#pragma unroll
        for (int j = 0; j < KB; ++j) lv[j] = (j < kw) ? A[r + (int64_t)(kb + j) * n] : T(0);
#pragma unroll
        for (int j = 0; j < KB; ++j)
          if (j < kw)
#pragma unroll
            for (int c = 0; c < NC; ++c) x[q][c] -= lv[j] * sX[j][c];
      }
    }
    __syncthreads();
  }
  // backward: U X = Y
  for (int kb = ((n - 1) / KB) * KB; kb >= 0; kb -= KB) {
    const int kw = min(KB, n - kb);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r >= kb && r < kb + kw)
#pragma unroll
        for (int c = 0; c < NC; ++c) sX[r - kb][c] = x[q][c];
    }
    for (int e = tid; e < kw * kw; e += NT) {
      const int i = e % kw, j = e / kw;
      sD[i][j] = A[(kb + i) + (int64_t)(kb + j) * n];
    }
    __syncthreads();
    if (tid < 32 * NC) {
      const int i = tid & 31, c = tid >> 5, base = tid & 32;
      T y = (i < kw) ? sX[i][c] : T(0);
      for (int j = kw - 1; j >= 0; --j) {
        if (i == j) y = y / sD[j][j];
        const T yj = __shfl(y, base + j, WAVE);
        if (i < j) y -= sD[i][j] * yj;
      }
      if (i < kw) sX[i][c] = y;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r >= kb && r < kb + kw) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[q][c] = sX[r - kb][c];
      } else if (r < kb) {
        T uv[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) uv[j] = (j < kw) ? A[r + (int64_t)(kb + j) * n] : T(0);
#pragma unroll
        for (int j = 0; j < KB; ++j)
          if (j < kw)
#pragma unroll
            for (int c = 0; c < NC; ++c) x[q][c] -= uv[j] * sX[j][c];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + NT * q;
    if (r < n)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c0 + c < n) out[(c0 + c) + (int64_t)r * n] = x[q][c];
  }
}

}  // namespace

// Register panel for the tallest panel of the launch: the smallest workgroup
// shape (threads x rows per thread) that holds min(rows, register limit) rows.
// A panel of width NB too tall for the register file, factored as two halves
// of width NB/2 (each a register panel of 512 threads x R rows): half 1; its
// interchanges and unit-lower solve on half 2's top rows; half 2 minus the
// rank-NB/2 product; half 2; half 2's interchanges on half 1.  The result (factors
// and pivots of the NB columns) is that of the NB-wide panel.
template <typename T, int NT, int R>
void launch_panel_split(const LuBatch& b, T* A, int k, hipStream_t s) {
  constexpr int H = LU_NB / 2;
  hipLaunchKernelGGL((k_lu_panel_rot<T, H, NT, R>), dim3(b.count), dim3(NT), 0, s, A, b.off, b.dim, b.piv, b.poff,
                     b.info, k, b.pad);
  GDSW_LAUNCH_CHECK();
  if (b.max_n <= k + H) return;
  hipLaunchKernelGGL((k_lu_inner_swap_trsm<T, H>), dim3(b.count), dim3(64), 0, s, A, b.off, b.dim, b.piv, b.poff, k,
                     b.pad);
  GDSW_LAUNCH_CHECK();
  const int tm = (int)blocks_for(b.max_n - k - H, TILE);
  hipLaunchKernelGGL((k_lu_update<T, H>), dim3((unsigned)((int64_t)b.count * tm)), dim3(256), 0, s, A, b.off, b.dim,
                     k, 1, tm, 1, nullptr, b.count, b.pad, nullptr, nullptr);
  GDSW_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_lu_panel_rot<T, H, NT, R>), dim3(b.count), dim3(NT), 0, s, A, b.off, b.dim, b.piv, b.poff,
                     b.info, k + H, b.pad);
  GDSW_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_lu_swap_cols<T>), dim3(b.count, 1), dim3(64), 0, s, A, b.off, b.dim, b.piv, b.poff, k + H, H,
                     k, H, b.pad);
  GDSW_LAUNCH_CHECK();
}

// split: every matrix of the batch is held by the register panels at this step
// (none is left to k_lu_panel), so the half-width path may run on all of them.
// Size classes: every matrix's panel goes to the smallest full-width register
// panel that holds it (one launch per class, over a range of the batch sorted by
// decreasing order) instead of all to the variant of the tallest one, so the
// short panels run with fewer registers per lane and more workgroups per CU.
// Only while no panel of the step needs the half-width or memory paths.
template <typename T>
bool launch_panel_classes(const LuBatch& b, T* A, int k, int rows, hipStream_t s) {
  constexpr int NB = LU_NB;
  if (!b.order || !b.order_dims || rows > (sizeof(T) == 8 ? 768 : 2048)) return false;
  // order_dims: orders in decreasing order; matrices with n - k in (lo, hi] form one class
  auto first_above = [&](int64_t n_lim) {     // first position whose order is <= n_lim
    int lo = 0, hi = b.count;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (b.order_dims[mid] > n_lim) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  int lo_cap = 0;
  auto cls = [&](auto kern, int nt, int cap) {
    const int p0 = first_above((int64_t)k + cap);
    const int p1 = first_above((int64_t)k + lo_cap);
    lo_cap = cap;
    if (p1 > p0) {
      hipLaunchKernelGGL(kern, dim3(p1 - p0), dim3(nt), 0, s, A, b.off, b.dim, b.piv, b.poff, b.info, k, b.pad,
                         b.order, p0);
      GDSW_LAUNCH_CHECK();
    }
  };
  cls(k_lu_panel_rot<T, NB, 256, 1>, 256, 256);
  cls(k_lu_panel_rot<T, NB, 256, 2>, 256, 512);
  cls(k_lu_panel_rot<T, NB, 256, 3>, 256, 768);
  if constexpr (sizeof(T) == 4) {
    cls(k_lu_panel_rot<T, NB, 512, 2>, 512, 1024);
    cls(k_lu_panel_rot<T, NB, 512, 3>, 512, 1536);
    cls(k_lu_panel_rot<T, NB, 512, 4>, 512, 2048);
  }
  return true;
}

template <typename T>
void launch_panel_rot(const LuBatch& b, T* A, int k, int rows, bool split, hipStream_t s) {
  constexpr int NB = LU_NB;
  if (b.panel_classes && launch_panel_classes<T>(b, A, k, rows, s)) return;
#define GDSW_PANEL(NT, R)                                                                                       \
  if (rows <= NT * R) {                                                                                         \
    hipLaunchKernelGGL((k_lu_panel_rot<T, NB, NT, R>), dim3(b.count), dim3(NT), 0, s, A, b.off, b.dim, b.piv, \
                       b.poff, b.info, k, b.pad);                                                                      \
    GDSW_LAUNCH_CHECK();                                                                                        \
    return;                                                                                                     \
  }
  GDSW_PANEL(256, 1)
  GDSW_PANEL(256, 2)
  GDSW_PANEL(256, 3)
  if constexpr (sizeof(T) == 8) {
    // FP64 panels of 769..1536 rows: half-width register panels that leave room
    // for two (256 threads) or three (512 threads) wavefronts per SIMD
    if (split && rows <= 256 * 4) {
      launch_panel_split<T, 256, 4>(b, A, k, s);
      return;
    }
    if (split && rows <= 512 * 3) {
      launch_panel_split<T, 512, 3>(b, A, k, s);
      return;
    }
  }
  GDSW_PANEL(512, 2)
  GDSW_PANEL(512, 3)
  if constexpr (sizeof(T) == 8) {
    if (split && rows <= 512 * 4) {
      launch_panel_split<T, 512, 4>(b, A, k, s);
      return;
    }
    GDSW_PANEL(1024, 2)
  }
  if constexpr (sizeof(T) == 4) {
    GDSW_PANEL(512, 4)
    if (split && rows <= 512 * 6) {
      launch_panel_split<T, 512, 6>(b, A, k, s);
      return;
    }
    GDSW_PANEL(512, 6)
  }
#undef GDSW_PANEL
  throw Error(-1, "panel taller than the register panel");
}

void LuTiles::build(const int* dims, int count) {
  constexpr int NB = LU_NB;
  int max_n = 0;
  for (int i = 0; i < count; ++i) max_n = std::max(max_n, dims[i]);
  const int steps = (max_n + 2 * NB - 1) / (2 * NB);
  outer.assign((size_t)steps * (count + 1), 0);
  inner.assign((size_t)steps * (count + 1), 0);
  total_outer.assign(steps, 0);
  total_inner.assign(steps, 0);
  for (int st = 0; st < steps; ++st) {
    const int k = st * 2 * NB;
    int64_t* po = outer.data() + (size_t)st * (count + 1);
    int64_t* pi = inner.data() + (size_t)st * (count + 1);
    for (int i = 0; i < count; ++i) {
      const int mo = dims[i] - k - 2 * NB, mi = dims[i] - k - NB;
      const int64_t to = mo > 0 ? (int64_t)((mo + TILE - 1) / TILE) * ((mo + TILE - 1) / TILE) : 0;
      const int64_t ti = mi > 0 ? (int64_t)((mi + TILE - 1) / TILE) : 0;
      po[i + 1] = po[i] + to;
      pi[i + 1] = pi[i] + ti;
    }
    total_outer[st] = po[count];
    total_inner[st] = pi[count];
  }
}

// Largest grid of k_tall_panel_coop that can be resident at once on the current
// device (0 when cooperative launches are not supported); taller panels take
// the per-column launches.
template <typename T>
int tall_coop_max_groups() {
  static std::mutex mu;
  static int cached[64];
  static bool known[64];
  int dev = 0;
  GDSW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!known[dev]) {
    int coop = 0, cus = 0, per_cu = 0;
    GDSW_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    GDSW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GDSW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_tall_panel_coop<T>, TALL_T, 0));
    cached[dev] = coop ? cus * per_cu : 0;
    known[dev] = true;
  }
  return cached[dev];
}

template <typename T>
void lu_batched(const LuBatch& b, T* A, hipStream_t s) {
  constexpr int NB = LU_NB;
  T* ut = static_cast<T*>(b.ut);
  auto panel = [&](int k) {
    const int rows = b.max_n - k;
    const bool tall = rows > panel_reg_rows<T>();
    if (tall && b.count == 1 && b.tall_scratch) {
      // a single large matrix (the coarsest): the panel is spread over many workgroups
      const int n = b.max_n;
      const int jb = std::min(TALL_NB, n - k);
      const int G = (int)blocks_for(rows, TALL_T);
      TallBufs<T> B;
      char* base = static_cast<char*>(b.tall_scratch);
      const int Gm = (int)blocks_for(n, TALL_T);
      B.val = reinterpret_cast<double*>(base);
      B.idx = reinterpret_cast<int*>(base + 2 * Gm * sizeof(double));
      B.cand = reinterpret_cast<T*>(base + 2 * Gm * (sizeof(double) + sizeof(int)) + 64);
      B.rowj = B.cand + (size_t)2 * Gm * TALL_NB;
      int ld = lead_dim(n, b.pad);
      if (G <= tall_coop_max_groups<T>()) {
        int kk = k, nn = n, jj = jb, gg = G;
        T* AA = A;
        int* pv = b.piv;
        int* inf = b.info;
        void* args[] = {&AA, &ld, &nn, &kk, &jj, &gg, &B, &pv, &inf};
        GDSW_HIP(hipLaunchCooperativeKernel((const void*)k_tall_panel_coop<T>, dim3(G), dim3(TALL_T), args, 0, s));
        return;
      }
      hipLaunchKernelGGL((k_tall_first<T>), dim3(G), dim3(TALL_T), 0, s, A, ld, n, k, jb, G, B);
      GDSW_LAUNCH_CHECK();
      for (int j = k; j < k + jb; ++j) {
        hipLaunchKernelGGL((k_tall_step<T>), dim3(G), dim3(TALL_T), 0, s, A, ld, n, k, jb, j, G, B, b.piv, b.info);
        GDSW_LAUNCH_CHECK();
      }
      return;
    }
    if (tall) {
      hipLaunchKernelGGL((k_lu_panel<T, NB>), dim3(b.count), dim3(256), 0, s, A, b.off, b.dim, b.piv, b.poff,
                         b.info, k, b.pad);
      GDSW_LAUNCH_CHECK();
    }
    launch_panel_rot<T>(b, A, k, std::min(rows, panel_reg_rows<T>()), !tall && !b.full_panels, s);
  };
  // columns [k, k + 2NB): both sub-panels (the second brought up to date by the first), then the
  // interchanges of the step on the columns to their left
  auto block = [&](int k) {
    panel(k);
    if (b.max_n > k + NB) {
      hipLaunchKernelGGL((k_lu_inner_swap_trsm<T, NB>), dim3(b.count), dim3(64), 0, s, A, b.off, b.dim, b.piv, b.poff,
                         k, b.pad);
      GDSW_LAUNCH_CHECK();
      const int tm = (int)blocks_for(b.max_n - k - NB, TILE);
      const int st = k / (2 * NB);
      const int64_t grid = b.tiles_inner ? b.total_inner[st] : (int64_t)b.count * tm;
      if (grid > 0) {
        hipLaunchKernelGGL((k_lu_update<T, NB>), dim3((unsigned)grid), dim3(256), 0, s, A, b.off, b.dim, k, 1, tm, 1,
                           b.tiles_inner ? b.tiles_inner + (size_t)st * (b.count + 1) : nullptr, b.count, b.pad,
                           nullptr, nullptr);
        GDSW_LAUNCH_CHECK();
      }
      panel(k + NB);
    }
    hipLaunchKernelGGL((k_lu_outer_swap_left<T, NB>), dim3(b.count, blocks_for(k + NB, 64)), dim3(64), 0, s, A, b.off,
                       b.dim, b.piv, b.poff, k, b.pad);
    GDSW_LAUNCH_CHECK();
  };
  auto trsm = [&](int k, int rest, int swap, int ut_rows, int ut_row0, int ut_k0) {
    hipLaunchKernelGGL((k_lu_outer_swap_trsm<T, NB>), dim3(b.count, blocks_for(rest, TRSM_COLS)), dim3(TRSM_COLS), 0, s,
                       A, b.off, b.dim, b.piv, b.poff, k, b.pad, ut, swap, ut_rows, ut_row0, ut_k0);
    GDSW_LAUNCH_CHECK();
  };
  if (b.wide && ut) {
    // Pairs of 2NB-column steps with one rank-4NB trailing update per pair (half the
    // passes over the trailing matrix).  For the pair at k0: the first block; U12 of
    // its rows for every trailing column (scratch rows 0..2NB); the second block's
    // columns updated; the second block; its interchanges, its rows updated by the
    // first block and its U12 (scratch rows 2NB..4NB) on the columns beyond; then
    // A22 -= L21 U12 over the 4NB columns of the pair.
    const int64_t huge = 1 << 30;
    for (int k0 = 0; k0 < b.max_n; k0 += 4 * NB) {
      block(k0);
      const int rest_a = b.max_n - k0 - 2 * NB;
      if (rest_a <= 0) break;
      trsm(k0, rest_a, 1, 4 * NB, 0, k0);
      {
        const int tm = (int)blocks_for(rest_a, TILE);
        hipLaunchKernelGGL((k_lu_update_ut<T, 2 * NB>), dim3((unsigned)((int64_t)b.count * tm)), dim3(256), 0, s, A,
                           b.off, b.dim, k0, 2 * NB, (int)huge, 2 * NB, 4 * NB, 2 * NB, tm, 1, nullptr, b.count, b.pad,
                           static_cast<const T*>(ut), b.poff, 4 * NB, nullptr);
        GDSW_LAUNCH_CHECK();
      }
      block(k0 + 2 * NB);
      const int rest_b = b.max_n - k0 - 4 * NB;
      if (rest_b <= 0) break;
      hipLaunchKernelGGL((k_lu_swap_cols<T>), dim3(b.count, blocks_for(rest_b, 64)), dim3(64), 0, s, A, b.off, b.dim,
                         b.piv, b.poff, k0 + 2 * NB, 2 * NB, k0 + 4 * NB, rest_b, b.pad);
      GDSW_LAUNCH_CHECK();
      {
        const int tn = (int)blocks_for(rest_b, TILE);
        hipLaunchKernelGGL((k_lu_update_ut<T, 2 * NB>), dim3((unsigned)((int64_t)b.count * tn)), dim3(256), 0, s, A,
                           b.off, b.dim, k0, 2 * NB, 2 * NB, 4 * NB, -1, 2 * NB, 1, tn, nullptr, b.count, b.pad,
                           static_cast<const T*>(ut), b.poff, 4 * NB, nullptr);
        GDSW_LAUNCH_CHECK();
      }
      trsm(k0 + 2 * NB, rest_b, 0, 4 * NB, 2 * NB, k0);
      {
        const int t = (int)blocks_for(rest_b, TILE);
        const int st = k0 / (2 * NB) + 1;
        const int64_t grid = b.tiles_outer ? b.total_outer[st] : (int64_t)b.count * t * t;
        if (grid > 0) {
          if (b.step_masks) {
            hipLaunchKernelGGL((k_lu_step_masks<T>), dim3(b.count), dim3(256), 0, s, A, b.off, b.dim, k0, b.pad,
                               static_cast<const T*>(ut), b.poff, 4 * NB, b.step_masks);
            GDSW_LAUNCH_CHECK();
          }
          hipLaunchKernelGGL((k_lu_update_ut<T, 4 * NB>), dim3((unsigned)grid), dim3(256), 0, s, A, b.off, b.dim, k0,
                             4 * NB, (int)huge, 4 * NB, -1, 4 * NB, t, t,
                             b.tiles_outer ? b.tiles_outer + (size_t)st * (b.count + 1) : nullptr, b.count, b.pad,
                             static_cast<const T*>(ut), b.poff, 4 * NB,
                             static_cast<const unsigned long long*>(b.step_masks));
          GDSW_LAUNCH_CHECK();
        }
      }
    }
    return;
  }
  for (int k = 0; k < b.max_n; k += 2 * NB) {
    block(k);
    const int rest = b.max_n - k - 2 * NB;
    if (rest > 0) {
      trsm(k, rest, 1, 2 * NB, 0, k);
      const int t = (int)blocks_for(rest, TILE);
      const int st = k / (2 * NB);
      const int64_t grid = b.tiles_outer ? b.total_outer[st] : (int64_t)b.count * t * t;
      if (grid > 0) {
        hipLaunchKernelGGL((k_lu_update<T, NB>), dim3((unsigned)grid), dim3(256), 0, s, A, b.off, b.dim, k, 0, t, t,
                           b.tiles_outer ? b.tiles_outer + (size_t)st * (b.count + 1) : nullptr, b.count, b.pad,
                           static_cast<const T*>(ut), b.poff);
        GDSW_LAUNCH_CHECK();
      }
    }
  }
}

template <typename T>
void lu_solve_batched(const LuBatch& b, const T* A, T* X, const int64_t* xoff, const int* nrhs, int max_rhs,
                      hipStream_t s) {
  if (b.pad > 1) throw Error(-1, "lu_solve_batched: padded blocks are not supported");
  constexpr int NB = LU_NB;
  const unsigned rhsblocks = blocks_for(max_rhs, 64);
  hipLaunchKernelGGL((k_getrs_swap<T>), dim3(b.count, rhsblocks), dim3(64), 0, s, b.dim, b.piv, b.poff, X, xoff,
                     nrhs);
  GDSW_LAUNCH_CHECK();
  const int tn = (int)blocks_for(max_rhs, TILE);
  const int tm = (int)blocks_for(b.max_n, TILE);
  const int tiles = (tm > tn ? tm : tn);
  for (int k = 0; k < b.max_n; k += NB) {
    hipLaunchKernelGGL((k_getrs_diag<T, NB>), dim3(b.count, rhsblocks), dim3(64), 0, s, A, b.off, b.dim, X, xoff,
                       nrhs, k, 0);
    GDSW_LAUNCH_CHECK();
    if (b.max_n - k - NB > 0) {
      hipLaunchKernelGGL((k_gemm_update<T, NB>), dim3(b.count * tiles * tiles), dim3(256), 0, s, (T*)A, b.off,
                         b.dim, X, xoff, nrhs, k, 1, tiles);
      GDSW_LAUNCH_CHECK();
    }
  }
  const int last = ((b.max_n - 1) / NB) * NB;
  for (int k = last; k >= 0; k -= NB) {
    hipLaunchKernelGGL((k_getrs_diag<T, NB>), dim3(b.count, rhsblocks), dim3(64), 0, s, A, b.off, b.dim, X, xoff,
                       nrhs, k, 1);
    GDSW_LAUNCH_CHECK();
    if (k > 0) {
      hipLaunchKernelGGL((k_gemm_update<T, NB>), dim3(b.count * tiles * tiles), dim3(256), 0, s, (T*)A, b.off,
                         b.dim, X, xoff, nrhs, k, 2, tiles);
      GDSW_LAUNCH_CHECK();
    }
  }
}

bool lu_inverse_transposed(const double* LU, const int* perm, double* out, int n, hipStream_t s) {
  constexpr int NC = 8;
  const unsigned grid = blocks_for(n, NC);
#define GDSW_INV(R)                                                                                       \
  if (n <= 512 * R) {                                                                                     \
    hipLaunchKernelGGL((k_inverse_resident<double, R, NC>), dim3(grid), dim3(512), 0, s, LU, perm, out, n); \
    GDSW_LAUNCH_CHECK();                                                                                  \
    return true;                                                                                          \
  }
  GDSW_INV(1)
  GDSW_INV(2)
  GDSW_INV(4)
  GDSW_INV(8)
#undef GDSW_INV
  return false;
}

void lu_build_perm(const LuBatch& b, int* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_build_perm, dim3(b.count), dim3(256), 0, s, b.dim, b.piv, b.poff, perm);
  GDSW_LAUNCH_CHECK();
}

void lu_inverse_blocked(const LuBatch& b, const double* LU, const int* perm, double* X, int* scratch, int n,
                        hipStream_t s) {
  constexpr int NB = LU_NB, BB = 4 * LU_NB;
  const int tn = (int)blocks_for(n, TILE);
  int* pinv = scratch;
  int* lo = scratch + n;
  hipLaunchKernelGGL(k_inv_first_rows, dim3(blocks_for(n, 256)), dim3(256), 0, s, perm, n, pinv, lo, 0);
  GDSW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_inv_first_rows, dim3(blocks_for(tn, 256)), dim3(256), 0, s, perm, n, pinv, lo, 1);
  GDSW_LAUNCH_CHECK();
  set_identity<double>(X, n, s);
  const unsigned rhsblocks = blocks_for(n, 64);
  hipLaunchKernelGGL((k_getrs_swap<double>), dim3(1, rhsblocks), dim3(64), 0, s, b.dim, b.piv, b.poff, X, b.off, b.dim);
  GDSW_LAUNCH_CHECK();
  auto update = [&](int r0, int M, int kc, int kw, const int* lo_) {
    if (M <= 0 || kw <= 0) return;
    const int tm = (int)blocks_for(M, TILE);
    if (kw > NB)
      hipLaunchKernelGGL((k_inv_update<double, BB>), dim3((unsigned)tm * tn), dim3(256), 0, s, LU, X, n, r0, M, kc, kw,
                         tm, lo_);
    else
      hipLaunchKernelGGL((k_inv_update<double, NB>), dim3((unsigned)tm * tn), dim3(256), 0, s, LU, X, n, r0, M, kc, kw,
                         tm, lo_);
    GDSW_LAUNCH_CHECK();
  };
  auto diag = [&](int k, int upper) {
    hipLaunchKernelGGL((k_getrs_diag<double, NB>), dim3(1, rhsblocks), dim3(64), 0, s, LU, b.off, b.dim, X, b.off,
                       b.dim, k, upper);
    GDSW_LAUNCH_CHECK();
  };
  for (int kb = 0; kb < n; kb += BB) {
    const int e = std::min(kb + BB, n);
    for (int sb = kb; sb < e; sb += NB) {
      diag(sb, 0);
      update(sb + NB, e - (sb + NB), sb, std::min(NB, n - sb), lo);
    }
    update(e, n - e, kb, e - kb, lo);
  }
  const int last = ((n - 1) / BB) * BB;
  for (int kb = last; kb >= 0; kb -= BB) {
    const int e = std::min(kb + BB, n);
    for (int sb = ((e - 1 - kb) / NB) * NB + kb; sb >= kb; sb -= NB) {
      diag(sb, 1);
      update(kb, sb - kb, sb, std::min(NB, n - sb), nullptr);
    }
    update(0, kb, kb, e - kb, nullptr);
  }
}

size_t lu_tall_scratch_bytes(int n, int value_bytes) {
  const size_t Gm = blocks_for(n, TALL_T);
  return 2 * Gm * (sizeof(double) + sizeof(int)) + 64 + (2 * Gm + 2) * TALL_NB * (size_t)value_bytes + 256;
}

template void lu_batched<double>(const LuBatch&, double*, hipStream_t);
template void lu_batched<float>(const LuBatch&, float*, hipStream_t);
template void lu_solve_batched<double>(const LuBatch&, const double*, double*, const int64_t*, const int*, int,
                                       hipStream_t);
template void lu_solve_batched<float>(const LuBatch&, const float*, float*, const int64_t*, const int*, int,
                                      hipStream_t);

}  // namespace gdsw
