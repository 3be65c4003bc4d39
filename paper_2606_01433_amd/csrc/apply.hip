// Preconditioner apply, eq. (2.2): local solves R_i^T A_i^{-1} R_i, the
// ordered combination of overlapping values, the coarse restriction Phi^T r,
// the prolongation Phi y and the coarsest direct solve.
#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace gdsw {

namespace {

constexpr int PW = 64;   // triangle / panel width of the blocked substitution

// ---------------------------------------------------------------------------
// Local solves w_i = A_i^{-1} R_i r with the pivoted LU stored in place.
// Forward substitution with unit L, then backward with U, in 64-wide panels:
// the diagonal triangle is solved by one wave (lane j's value is broadcast with
// readlane), then the panel is applied to the remaining rows as a GEMV in
// row-outer order (each thread streams its row's 64 panel entries with the
// loads in flight together).  The gathered right-hand side lives in LDS.
//
// NW wavefronts per matrix share the GEMV rows (8 by default; the autotuner may
// pick 2 or 4).  With 8, a panel row is loaded in two phases of 32 columns
// (half the registers: four waves per SIMD instead of three) into the same
// 64-term accumulation, so every choice gives bit-identical results.
// Matrices are visited largest first (`order`), so the big ones do not form
// the tail.  FIRST only separates the level-1 launch from deeper levels in
// profiles.  Columns are stored with leading dimension lead_dim(n, pad).
//
// Register discipline: a panel row is addressed through one running 64-bit
// offset made opaque to the optimizer after each step, and the per-column lane
// masks of the triangles are formed next to their use from an opaque copy of
// the lane index; otherwise the compiler hoists 64 column offsets and 64 lane
// masks into scalar registers and spills them (half of a lone matrix's time).
// FULL = false handles the one ragged panel of a matrix (pw < 64 columns).
// ---------------------------------------------------------------------------
template <typename T, int NPH, bool FULL>
__device__ __forceinline__ void ls_row_update(const T* __restrict__ A, int ld, T* x, int row, int q0, int pw) {
  constexpr int H = PW / NPH;
  T acc = T(0);
#pragma unroll
  for (int h = 0; h < NPH; ++h) {
    int64_t o = row + (int64_t)(q0 + h * H) * ld;
    if (h > 0) asm volatile("" : "+v"(o) : "v"(acc));   // phase h loads after phase h-1 (register budget)
    T v[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      v[j] = (FULL || h * H + j < pw) ? ld_stream(A + o) : T(0);
      o += ld;
      asm volatile("" : "+v"(o));
    }
#pragma unroll
    for (int j = 0; j < H; ++j) acc += v[j] * x[q0 + (FULL ? h * H + j : min(h * H + j, pw - 1))];
  }
  x[row] -= acc;
}

// Unit-lower triangle of rows/columns [q0, q0 + pw) solved in place in x by one wave.
// Lanes at or past pw address row q0 (valid memory) and are masked out.
template <typename T, int NPH, bool FULL>
__device__ __forceinline__ void ls_tri_lower(const T* __restrict__ A, int ld, T* x, int q0, int pw, int lane) {
  constexpr int H = PW / NPH;
  const bool ok = FULL || lane < pw;
  const int row = ok ? q0 + lane : q0;
  const int lj = ok ? lane : 0;
  T xv = ok ? x[row] : T(0);
#pragma unroll
  for (int h = 0; h < NPH; ++h) {
    if (!(FULL || h * H < pw)) continue;
    int64_t o = row + (int64_t)(q0 + h * H) * ld;
    if (h > 0) asm volatile("" : "+v"(o) : "v"(xv));
    T d[H];   // strictly lower part only: the other lanes fetch nothing
#pragma unroll
    for (int j = 0; j < H; ++j) {
      int l = lj;
      asm volatile("" : "+v"(l));
      d[j] = (h * H + j < l) ? ld_stream(A + o) : T(0);
      o += ld;
      asm volatile("" : "+v"(o));
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int jj = h * H + j;
      if (FULL || jj < pw) xv -= d[j] * lane_value(xv, jj);
    }
  }
  if (ok) x[row] = xv;
}

// Upper triangle (non-unit diagonal) of rows/columns [q0, q0 + pw), one wave: the value of
// column jj is broadcast as x_jj * (1 / U_jj); each lane scales its own value once at the end.
template <typename T, int NPH, bool FULL>
__device__ __forceinline__ void ls_tri_upper(const T* __restrict__ A, int ld, T* x, int q0, int pw, int lane) {
  constexpr int H = PW / NPH;
  const bool ok = FULL || lane < pw;
  const int row = ok ? q0 + lane : q0;
  const T rd = ok ? T(1) / A[row + (int64_t)row * ld] : T(0);
  const int lj = ok ? lane : PW;
  T xv = ok ? x[row] : T(0);
#pragma unroll
  for (int h = NPH - 1; h >= 0; --h) {
    if (!(FULL || h * H < pw)) continue;
    int64_t o = row + (int64_t)(q0 + h * H) * ld;
    if (h < NPH - 1) asm volatile("" : "+v"(o) : "v"(xv));
    T d[H];   // strictly upper part within the pw columns only
#pragma unroll
    for (int j = 0; j < H; ++j) {
      int l = lj;
      asm volatile("" : "+v"(l));
      d[j] = (h * H + j > l && (FULL || h * H + j < pw)) ? ld_stream(A + o) : T(0);
      o += ld;
      asm volatile("" : "+v"(o));
    }
#pragma unroll
    for (int j = H - 1; j >= 0; --j) {
      const int jj = h * H + j;
      if (FULL || jj < pw) xv -= d[j] * (lane_value(xv, jj) * lane_value(rd, jj));
    }
  }
  xv *= rd;
  if (ok) x[row] = xv;
}

template <typename T, bool FIRST, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 4 : 1))) void k_local_solve_wg(
    const int* __restrict__ order, const int64_t* __restrict__ dom_ptr, const int* __restrict__ gidx,
    const int64_t* __restrict__ blk_off, const T* __restrict__ blocks, const double* __restrict__ r,
    double* __restrict__ w, int pad, const int64_t* __restrict__ moff, const unsigned long long* __restrict__ tmask) {
  constexpr int NT = 64 * NW;
  constexpr int NPH = NW == 8 ? 2 : 1;
  extern __shared__ unsigned char smem_raw[];
  T* x = reinterpret_cast<T*>(smem_raw);
  const int i = order[blockIdx.x];
  const int64_t base = dom_ptr[i];
  const int n = (int)(dom_ptr[i + 1] - base);
  const T* A = blocks + blk_off[i];
  const int ld = lead_dim(n, pad);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // tile masks of this block: nw words per 64-column panel, bit q of word (p, q / 64) set when
  // the 64-row tile q of panel p holds a nonzero
  const unsigned long long* M = tmask + moff[i];
  const int nt = (n + PW - 1) / PW, nw = (nt + 63) >> 6;
  for (int a = tid; a < n; a += NT) x[a] = (T)r[gidx[base + a]];
  __syncthreads();
  for (int p0 = 0; p0 < n; p0 += PW) {
    const int pw = min(PW, n - p0);
    const int p = p0 / PW;
    if (wid == 0) {
      if (pw == PW) ls_tri_lower<T, NPH, true>(A, ld, x, p0, PW, lane);
      else ls_tri_lower<T, NPH, false>(A, ld, x, p0, pw, lane);
    }
    __syncthreads();
    // the nonzero row tiles below the panel (none below a ragged last panel), dealt to the
    // wavefronts in turn
    int k = 0;
    for (int wi = (p + 1) >> 6; wi < nw; ++wi) {
      unsigned long long bits = M[(int64_t)p * nw + wi];
      if (wi == (p + 1) >> 6) bits &= ~0ull << ((p + 1) & 63);
      for (; bits; ++k) {
        const int q = wi * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        const int rr = q * PW + lane;
        if ((k & (NW - 1)) == wid && rr < n) ls_row_update<T, NPH, true>(A, ld, x, rr, p0, PW);
      }
    }
    __syncthreads();
  }
  for (int p0 = ((n - 1) / PW) * PW; p0 >= 0; p0 -= PW) {
    const int pw = min(PW, n - p0);
    const int p = p0 / PW;
    if (wid == 0) {
      if (pw == PW) ls_tri_upper<T, NPH, true>(A, ld, x, p0, PW, lane);
      else ls_tri_upper<T, NPH, false>(A, ld, x, p0, pw, lane);
    }
    __syncthreads();
    // the nonzero row tiles above the panel (all their rows lie above it)
    int k = 0;
    for (int wi = 0; wi <= (p >> 6); ++wi) {
      unsigned long long bits = M[(int64_t)p * nw + wi];
      if (wi == (p >> 6)) bits &= (1ull << (p & 63)) - 1ull;
      for (; bits; ++k) {
        const int q = wi * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        if ((k & (NW - 1)) != wid) continue;
        const int rr = q * PW + lane;
        if (pw == PW) ls_row_update<T, NPH, true>(A, ld, x, rr, p0, PW);
        else ls_row_update<T, NPH, false>(A, ld, x, rr, p0, pw);
      }
    }
    __syncthreads();
  }
  for (int a = tid; a < n; a += NT) w[base + a] = (double)x[a];
}

// ---------------------------------------------------------------------------
// Local solves of KC right-hand sides at once (the same factor streamed once
// for all of them).  Same blocked substitution as k_local_solve_wg, with the
// gathered right-hand sides in LDS row by row (x[a * KC + s]): the diagonal
// triangles take each right-hand side's operations in the single kernel's
// order, the panel updates run on MFMA (sums of four products per step, so a
// column agrees with the single-right-hand-side result to rounding, not bit for
// bit).  Right-hand side s of the chunk is R[s * ldr + g]; the local solutions go
// to W[s * ldw + position].
// ---------------------------------------------------------------------------
// The diagonal triangles of the chunk, one right-hand side s per wave: the
// operations of ls_tri_lower / ls_tri_upper on column s of the LDS block (same
// order, so each column equals the single-right-hand-side result), KC waves
// side by side.  The factor's triangle is read with plain loads: the KC waves
// read the same tile.
template <typename T, int NPH, bool FULL, int KC>
__device__ __forceinline__ void lsm_tri_lower_one(const T* __restrict__ A, int ld, T* x, int q0, int pw, int lane,
                                                  int s) {
  constexpr int H = PW / NPH;
  const bool ok = FULL || lane < pw;
  const int row = ok ? q0 + lane : q0;
  const int lj = ok ? lane : 0;
  T xv = ok ? x[row * KC + s] : T(0);
#pragma unroll
  for (int h = 0; h < NPH; ++h) {
    if (!(FULL || h * H < pw)) continue;
    int64_t o = row + (int64_t)(q0 + h * H) * ld;
    if (h > 0) asm volatile("" : "+v"(o) : "v"(xv));
    T d[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      int l = lj;
      asm volatile("" : "+v"(l));
      d[j] = (h * H + j < l) ? A[o] : T(0);
      o += ld;
      asm volatile("" : "+v"(o));
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int jj = h * H + j;
      if (FULL || jj < pw) xv -= d[j] * lane_value(xv, jj);
    }
  }
  if (ok) x[row * KC + s] = xv;
}

template <typename T, int NPH, bool FULL, int KC>
__device__ __forceinline__ void lsm_tri_upper_one(const T* __restrict__ A, int ld, T* x, int q0, int pw, int lane,
                                                  int s) {
  constexpr int H = PW / NPH;
  const bool ok = FULL || lane < pw;
  const int row = ok ? q0 + lane : q0;
  const T rd = ok ? T(1) / A[row + (int64_t)row * ld] : T(0);
  const int lj = ok ? lane : PW;
  T xv = ok ? x[row * KC + s] : T(0);
#pragma unroll
  for (int h = NPH - 1; h >= 0; --h) {
    if (!(FULL || h * H < pw)) continue;
    int64_t o = row + (int64_t)(q0 + h * H) * ld;
    if (h < NPH - 1) asm volatile("" : "+v"(o) : "v"(xv));
    T d[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      int l = lj;
      asm volatile("" : "+v"(l));
      d[j] = (h * H + j > l && (FULL || h * H + j < pw)) ? A[o] : T(0);
      o += ld;
      asm volatile("" : "+v"(o));
    }
#pragma unroll
    for (int j = H - 1; j >= 0; --j) {
      const int jj = h * H + j;
      if (FULL || jj < pw) xv -= d[j] * (lane_value(xv, jj) * lane_value(rd, jj));
    }
  }
  if (ok) x[row * KC + s] = xv * rd;
}

// The panel update of the chunk as a small GEMM on the matrix cores:
// x[r, s] -= sum_k A[r, q0 + k] x[q0 + k, s] for the rows r < r1 of the 64-row
// tiles t0 <= q < t1 whose bit is set in the panel's masks M (the other tiles of
// the panel are zero), k < pw, s < KC.  Waves take 16-row blocks in turn; one
// 16x16x4 MFMA per four panel columns, its 16 output columns the right-hand
// sides (KC of them used), so each lane reads one right-hand-side value per MFMA
// from LDS instead of one broadcast per FMA.  Operand layout as in the LU's MFMA tiles (transposed
// product: lane (li, lk) feeds row li / column li and k = 4 step + lk, and
// holds C[row li][column mfma_col(lk, q)]).
template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lk, int q) { return lk + 4 * q; }
};
template <> struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lk, int q) { return 4 * lk + q; }
};

template <typename T, int KC, int NW>
__device__ __forceinline__ void lsm_update_mfma(const T* __restrict__ A, int ld, T* x, const unsigned long long* M,
                                                int t0, int t1, int r1, int q0, int pw, int wid, int lane) {
  typedef typename Mma<T>::v4 v4;
  const int li = lane & 15, lk = lane >> 4;
  // the panel's right-hand-side operands do not change during the update: read them once
  T b[PW / 4];
#pragma unroll
  for (int st = 0; st < PW / 4; ++st) {
    const int k = 4 * st + lk;
    b[st] = (li < KC && k < pw) ? x[(q0 + k) * KC + li] : T(0);
  }
  // the 16-row blocks of the nonzero 64-row tiles t0 <= q < t1, dealt to the wavefronts in turn
  int k = 0;
  for (int wi = t0 >> 6; t0 < t1 && wi <= (t1 - 1) >> 6; ++wi) {
    unsigned long long bits = M[wi];
    if (wi == t0 >> 6) bits &= ~0ull << (t0 & 63);
    if (wi == (t1 - 1) >> 6 && ((t1 - 1) & 63) < 63) bits &= (1ull << (((t1 - 1) & 63) + 1)) - 1ull;
    while (bits) {
      const int q = wi * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      for (int sb = 0; sb < PW / 16; ++sb, ++k) {
        const int rb = q * PW + 16 * sb;
        if ((k & (NW - 1)) != wid || rb >= r1) continue;
        const int row = rb + li;
        const bool in = row < r1;
        T a[PW / 4];
        int64_t o = (int64_t)(in ? row : rb) + (int64_t)(q0 + lk) * ld;
        asm volatile("" : "+v"(o));
#pragma unroll
        for (int st = 0; st < PW / 4; ++st) {
          a[st] = (in && 4 * st + lk < pw) ? ld_stream(A + o) : T(0);
          o += 4 * (int64_t)ld;
          asm volatile("" : "+v"(o));
        }
        v4 acc = v4{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < PW / 4; ++st) acc = Mma<T>::mac(b[st], a[st], acc);
        if (in) {
#pragma unroll
          for (int q2 = 0; q2 < 4; ++q2) {
            const int c = Mma<T>::col(lk, q2);
            if (c < KC) x[row * KC + c] -= acc[q2];
          }
        }
      }
    }
  }
}

template <typename T, int KC>
__global__ __launch_bounds__(512) void k_local_solve_multi(const int* __restrict__ order,
                                                           const int64_t* __restrict__ dom_ptr,
                                                           const int* __restrict__ gidx,
                                                           const int64_t* __restrict__ blk_off,
                                                           const T* __restrict__ blocks, const double* __restrict__ R,
                                                           int64_t ldr, double* __restrict__ W, int64_t ldw, int kk,
                                                           int pad, const int64_t* __restrict__ moff,
                                                           const unsigned long long* __restrict__ tmask) {
  constexpr int NW = 8, NT = 64 * NW, NPH = 2;
  extern __shared__ unsigned char smem_raw[];
  T* x = reinterpret_cast<T*>(smem_raw);
  const int i = order[blockIdx.x];
  const int64_t base = dom_ptr[i];
  const int n = (int)(dom_ptr[i + 1] - base);
  const T* A = blocks + blk_off[i];
  const int ld = lead_dim(n, pad);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const unsigned long long* M = tmask + moff[i];   // nonzero-tile masks (see k_tile_mask)
  const int nt = (n + PW - 1) / PW, nw = (nt + 63) >> 6;
  for (int a = tid; a < n; a += NT) {
    const int g = gidx[base + a];
#pragma unroll
    for (int s = 0; s < KC; ++s) x[a * KC + s] = s < kk ? (T)R[s * ldr + g] : T(0);
  }
  __syncthreads();
  for (int p0 = 0; p0 < n; p0 += PW) {
    const int pw = min(PW, n - p0);
    if (wid < KC) {
      if (pw == PW) lsm_tri_lower_one<T, NPH, true, KC>(A, ld, x, p0, PW, lane, wid);
      else lsm_tri_lower_one<T, NPH, false, KC>(A, ld, x, p0, pw, lane, wid);
    }
    __syncthreads();
    lsm_update_mfma<T, KC, NW>(A, ld, x, M + (int64_t)(p0 / PW) * nw, p0 / PW + 1, nt, n, p0, pw, wid,
                               lane);   // rows below the panel
    __syncthreads();
  }
  for (int p0 = ((n - 1) / PW) * PW; p0 >= 0; p0 -= PW) {
    const int pw = min(PW, n - p0);
    if (wid < KC) {
      if (pw == PW) lsm_tri_upper_one<T, NPH, true, KC>(A, ld, x, p0, PW, lane, wid);
      else lsm_tri_upper_one<T, NPH, false, KC>(A, ld, x, p0, pw, lane, wid);
    }
    __syncthreads();
    lsm_update_mfma<T, KC, NW>(A, ld, x, M + (int64_t)(p0 / PW) * nw, 0, p0 / PW, p0, p0, pw, wid,
                               lane);   // rows above the panel
    __syncthreads();
  }
  for (int a = tid; a < n; a += NT) {
#pragma unroll
    for (int s = 0; s < KC; ++s)
      if (s < kk) W[s * ldw + base + a] = (double)x[a * KC + s];
  }
}

__global__ void k_scatter_sum(int64_t n, const int64_t* __restrict__ sc_ptr, const int* __restrict__ sc_pos,
                              const double* __restrict__ w, double* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (!sc_ptr) {                       // restricted: one position per dof (still a sum into zero)
    z[g] = 0.0 + w[sc_pos[g]];
    return;
  }
  double s = 0.0;
  for (int64_t k = sc_ptr[g]; k < sc_ptr[g + 1]; ++k) s += w[sc_pos[k]];
  z[g] = s;
}

// rc[c] = sum of r over the interface dofs of column c + Phi_I columns of the parts holding c.
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(int n_coarse, const int64_t* __restrict__ col_ptr,
                                                  const int* __restrict__ col_dofs, const int64_t* __restrict__ cp_ptr,
                                                  const int* __restrict__ cp_part, const int* __restrict__ cp_lc,
                                                  const int64_t* __restrict__ int_ptr, const int* __restrict__ inter,
                                                  const int64_t* __restrict__ phi_off, const T* __restrict__ phi,
                                                  const double* __restrict__ r, double* __restrict__ rc) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n_coarse) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int64_t k = col_ptr[c] + lane; k < col_ptr[c + 1]; k += 64) s += r[col_dofs[k]];
  // the parts holding c: lane t fetches entry t's part data, then the parts are
  // visited in order with their data broadcast from the owning lane
  const int64_t t0 = cp_ptr[c], t1 = cp_ptr[c + 1];
  for (int64_t tb = t0; tb < t1; tb += 64) {
    const int cnt = (int)min((int64_t)64, t1 - tb);
    int64_t ib = 0, poff = 0;
    int nI = 0;
    if (lane < cnt) {
      const int i = cp_part[tb + lane];
      ib = int_ptr[i];
      nI = (int)(int_ptr[i + 1] - ib);
      poff = phi_off[i] + (int64_t)cp_lc[tb + lane] * nI;
    }
    for (int t = 0; t < cnt; ++t) {
      const int64_t ibt = ((int64_t)lane_value((int)(ib >> 32), t) << 32) | (unsigned int)lane_value((int)ib, t);
      const int64_t pot = ((int64_t)lane_value((int)(poff >> 32), t) << 32) | (unsigned int)lane_value((int)poff, t);
      const int nIt = lane_value(nI, t);
      const T* ph = phi + pot;
      const int* I = inter + ibt;
      for (int a = lane; a < nIt; a += 64) s += (double)ld_stream(ph + a) * r[I[a]];
    }
  }
  s = wave_sum(s);
  if (lane == 0) rc[c] = s;
}

// z[g] += y[col(g)] for the interface dofs (Phi_Gamma has a single one per row).
__global__ void k_prolong_gamma(int64_t count, const int* __restrict__ gdofs, const int* __restrict__ dof_gcol,
                                const double* __restrict__ y, double* __restrict__ z) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int g = gdofs[k];
  z[g] += y[dof_gcol[g]];
}

// z[I_i[a]] += sum_c Phi_I[a, c] y[col_i(c)], one workgroup per part, the part's
// coarse values staged in LDS (interior dofs belong to one part only).
template <typename T>
__global__ __launch_bounds__(128) void k_prolong_interior(const int64_t* __restrict__ int_ptr,
                                                          const int* __restrict__ inter,
                                                          const int64_t* __restrict__ pc_ptr,
                                                          const int* __restrict__ pcols,
                                                          const int64_t* __restrict__ phi_off,
                                                          const T* __restrict__ phi, const double* __restrict__ y,
                                                          double* __restrict__ z) {
  extern __shared__ double ys[];
  const int i = blockIdx.x;
  const int64_t ib = int_ptr[i];
  const int nI = (int)(int_ptr[i + 1] - ib);
  const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
  const int* pc = pcols + pc_ptr[i];
  for (int c = threadIdx.x; c < m; c += blockDim.x) ys[c] = y[pc[c]];
  __syncthreads();
  const T* ph = phi + phi_off[i];
  for (int a = threadIdx.x; a < nI; a += blockDim.x) {
    double p = 0.0;
    for (int c = 0; c < m; ++c) p += (double)ld_stream(ph + a + (int64_t)c * nI) * ys[c];
    z[inter[ib + a]] += p;
  }
}

// y[r] = sum_c Ainv[r, c] x[c] with the inverse stored transposed (row r contiguous): one wave per row,
// four independent partial sums per lane (columns c, c + 64, c + 128, c + 192 of each 256-column
// stretch) so that four loads per lane are in flight, combined in a fixed order.
__global__ __launch_bounds__(256) void k_gemv_rows(int n, const double* __restrict__ AT, const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const int lane = threadIdx.x & 63;
  const double* row = AT + (int64_t)r * n;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = lane;
  for (; c + 192 < n; c += 256) {
    const double a0 = ld_stream(row + c), a1 = ld_stream(row + c + 64), a2 = ld_stream(row + c + 128),
                 a3 = ld_stream(row + c + 192);
    const double x0 = x[c], x1 = x[c + 64], x2 = x[c + 128], x3 = x[c + 192];
    s0 += a0 * x0;
    s1 += a1 * x1;
    s2 += a2 * x2;
    s3 += a3 * x3;
  }
  for (; c < n; c += 64) s0 += ld_stream(row + c) * x[c];
  double s = (s0 + s1) + (s2 + s3);
  s = wave_sum(s);
  if (lane == 0) y[r] = s;
}

__global__ void k_transpose(int n, const double* __restrict__ A, double* __restrict__ AT) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = bx + threadIdx.x, c = by + k;
    if (r < n && c < n) t[k][threadIdx.x] = A[r + (int64_t)c * n];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = by + threadIdx.x, c = bx + k;       // AT[r + c n] = A[c + r n]
    if (r < n && c < n) AT[r + (int64_t)c * n] = t[threadIdx.x][k];
  }
}

}  // namespace

// LDS a workgroup may use on the current device (160 KiB on gfx950), cached per device.
size_t lds_per_block() {
  static std::mutex mu;
  static size_t cached[64];
  int dev = 0;
  GDSW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return 64 * 1024;
  std::lock_guard<std::mutex> lk(mu);
  if (!cached[dev]) {
    int v = 0;
    GDSW_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    cached[dev] = v > 0 ? (size_t)v : 64 * 1024;
  }
  return cached[dev];
}

// Which 64 x 64 tiles of the stored LU factors hold a nonzero: with nt = ceil(n_i / 64) tiles per
// side and nw = ceil(nt / 64) words per panel, bit q % 64 of tmask[moff[i] + p nw + q / 64] is set
// when rows [64 q, 64 q + 64) x columns [64 p, 64 p + 64) of block i (q != p) have a nonzero entry
// (q > p: the unit-lower factor, q < p: the upper one).  The substitution skips the other tiles:
// their products are exact zeros, so its result is unchanged.  tmask must be zeroed beforehand.
// kept[0] += the elements the substitution then reads (diagonal tiles and nonzero off-diagonal
// tiles).  One workgroup per block; every element is read once.
template <typename T>
__global__ __launch_bounds__(512) void k_tile_mask(const int64_t* __restrict__ dom_ptr,
                                                   const int64_t* __restrict__ blk_off, const T* __restrict__ blocks,
                                                   int pad, const int64_t* __restrict__ moff,
                                                   unsigned long long* __restrict__ tmask,
                                                   unsigned long long* __restrict__ kept) {
  __shared__ unsigned long long cnt;
  const int i = blockIdx.x;
  const int n = (int)(dom_ptr[i + 1] - dom_ptr[i]);
  unsigned long long* M = tmask + moff[i];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nt = (n + PW - 1) / PW, nw = (nt + 63) >> 6;
  if (tid == 0) cnt = 0ull;
  __syncthreads();
  const T* A = blocks + blk_off[i];
  const int ld = lead_dim(n, pad);
  for (int64_t t = wid; t < (int64_t)nt * nt; t += 8) {
    const int q = (int)(t / nt), p = (int)(t - (int64_t)q * nt);
    if (q == p) continue;
    const int row = q * PW + lane;
    const int c0 = p * PW, c1 = min(n, c0 + PW);
    bool nz = false;
    if (row < n) {
      int64_t o = row + (int64_t)c0 * ld;
#pragma unroll 16
      for (int c = c0; c < c1; ++c) {
        nz |= ld_stream(A + o) != T(0);
        o += ld;
      }
    }
    if (__any(nz) && lane == 0) {
      atomicOr(M + (int64_t)p * nw + (q >> 6), 1ull << (q & 63));
      atomicAdd(&cnt, (unsigned long long)(min(n, q * PW + PW) - q * PW) * (unsigned long long)(c1 - c0));
    }
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long diag = 0;
    for (int p = 0; p < nt; ++p) {
      const unsigned long long wp = (unsigned long long)min(PW, n - p * PW);
      diag += wp * wp;
    }
    atomicAdd(kept, cnt + diag);
  }
}

template <typename T>
void tile_masks(int nparts, const int64_t* dom_ptr, const int64_t* blk_off, const T* blocks, int pad,
                const int64_t* moff, unsigned long long* tmask, unsigned long long* kept, hipStream_t s) {
  if (nparts == 0) return;
  hipLaunchKernelGGL((k_tile_mask<T>), dim3(nparts), dim3(512), 0, s, dom_ptr, blk_off, blocks, pad, moff, tmask,
                     kept);
  GDSW_LAUNCH_CHECK();
}

template <typename T>
void local_solves(int nparts, int max_n, const int* order, const int64_t* dom_ptr, const int* gidx,
                  const int64_t* blk_off, const T* blocks, int pad, const int64_t* moff,
                  const unsigned long long* tmask, const double* r, double* w, bool first_level, int waves,
                  hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (nparts == 0) return;
  const size_t lds = (size_t)max_n * sizeof(T);
  if (lds > lds_per_block()) throw Error(-1, "local block too large for the LDS-resident right-hand side");
  if (waves != 2 && waves != 4 && waves != 8) throw Error(-1, "local solves: waves per matrix must be 2, 4 or 8");
  // with events, the dispatch itself records its start and end (exact kernel duration)
#define GDSW_LS(F, NW)                                                                                          \
  do {                                                                                                          \
    if (ev_start)                                                                                               \
      hipExtLaunchKernelGGL((k_local_solve_wg<T, F, NW>), dim3(nparts), dim3(64 * NW), lds, s, ev_start, ev_stop, \
                            0, order, dom_ptr, gidx, blk_off, blocks, r, w, pad, moff, tmask);                  \
    else                                                                                                        \
      hipLaunchKernelGGL((k_local_solve_wg<T, F, NW>), dim3(nparts), dim3(64 * NW), lds, s, order, dom_ptr,     \
                         gidx, blk_off, blocks, r, w, pad, moff, tmask);                                        \
  } while (0)
  if (first_level) {
    if (waves == 2) GDSW_LS(true, 2);
    else if (waves == 4) GDSW_LS(true, 4);
    else GDSW_LS(true, 8);
  } else {
    if (waves == 2) GDSW_LS(false, 2);
    else if (waves == 4) GDSW_LS(false, 4);
    else GDSW_LS(false, 8);
  }
#undef GDSW_LS
  GDSW_LAUNCH_CHECK();
}

int local_solves_multi_chunk(int max_n, int value_bytes) {
  const size_t per = (size_t)max_n * value_bytes;   // LDS bytes per right-hand side
  const size_t cap = lds_per_block();
  if (per * 8 <= cap) return 8;
  if (per * 4 <= cap) return 4;
  if (per * 2 <= cap) return 2;
  return 1;
}

template <typename T>
void local_solves_multi(int nparts, int max_n, const int* order, const int64_t* dom_ptr, const int* gidx,
                        const int64_t* blk_off, const T* blocks, int pad, const int64_t* moff,
                        const unsigned long long* tmask, const double* R, int64_t ldr, double* W, int64_t ldw, int k,
                        hipStream_t s) {
  if (nparts == 0 || k <= 0) return;
  const int kc = local_solves_multi_chunk(max_n, sizeof(T));
  if ((size_t)max_n * sizeof(T) > lds_per_block())
    throw Error(-1, "local block too large for the LDS-resident right-hand sides");
  for (int s0 = 0; s0 < k; s0 += kc) {
    const int kk = std::min(kc, k - s0);
    const double* Rs = R + (int64_t)s0 * ldr;
    double* Ws = W + (int64_t)s0 * ldw;
    const size_t lds = (size_t)max_n * sizeof(T) * kc;
#define GDSW_LSM(KC)                                                                                              \
  hipLaunchKernelGGL((k_local_solve_multi<T, KC>), dim3(nparts), dim3(512), lds, s, order, dom_ptr, gidx, blk_off, \
                     blocks, Rs, ldr, Ws, ldw, kk, pad, moff, tmask)
    if (kc == 8) GDSW_LSM(8);
    else if (kc == 4) GDSW_LSM(4);
    else if (kc == 2) GDSW_LSM(2);
    else GDSW_LSM(1);
#undef GDSW_LSM
    GDSW_LAUNCH_CHECK();
  }
}

void scatter_sum(int64_t n, const int64_t* sc_ptr, const int* sc_pos, const double* w, double* z, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_sum, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, sc_ptr, sc_pos, w, z);
  GDSW_LAUNCH_CHECK();
}

template <typename T>
void restrict_phi(int n_coarse, const int64_t* col_ptr, const int* col_dofs, const int64_t* cp_ptr,
                  const int* cp_part, const int* cp_lc, const int64_t* int_ptr, const int* inter,
                  const int64_t* phi_off, const T* phi, const double* r, double* rc, hipStream_t s) {
  hipLaunchKernelGGL((k_restrict<T>), dim3(blocks_for(n_coarse, 4)), dim3(256), 0, s, n_coarse, col_ptr, col_dofs,
                     cp_ptr, cp_part, cp_lc, int_ptr, inter, phi_off, phi, r, rc);
  GDSW_LAUNCH_CHECK();
}

template <typename T>
void prolong_add(int nparts, int max_m, int64_t n_gamma, const int* gdofs, const int* dof_gcol,
                 const int64_t* int_ptr, const int* inter, const int64_t* pc_ptr, const int* pcols,
                 const int64_t* phi_off, const T* phi, const double* y, double* z, hipStream_t s) {
  if (n_gamma > 0) {
    hipLaunchKernelGGL(k_prolong_gamma, dim3(blocks_for(n_gamma, 256)), dim3(256), 0, s, n_gamma, gdofs, dof_gcol, y,
                       z);
    GDSW_LAUNCH_CHECK();
  }
  if (nparts > 0) {
    hipLaunchKernelGGL((k_prolong_interior<T>), dim3(nparts), dim3(128), (size_t)max_m * sizeof(double), s, int_ptr,
                       inter, pc_ptr, pcols, phi_off, phi, y, z);
    GDSW_LAUNCH_CHECK();
  }
}

void transpose_square(int n, const double* A, double* AT, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3(blocks_for(n, 32), blocks_for(n, 32)), dim3(32, 8), 0, s, n, A, AT);
  GDSW_LAUNCH_CHECK();
}

void dense_gemv_rows(int n, const double* AT, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_rows, dim3(blocks_for(n, 4)), dim3(256), 0, s, n, AT, x, y);
  GDSW_LAUNCH_CHECK();
}

template void local_solves<double>(int, int, const int*, const int64_t*, const int*, const int64_t*,
                                   const double*, int, const int64_t*, const unsigned long long*, const double*,
                                   double*, bool, int, hipStream_t, hipEvent_t, hipEvent_t);
template void local_solves_multi<double>(int, int, const int*, const int64_t*, const int*, const int64_t*,
                                         const double*, int, const int64_t*, const unsigned long long*,
                                         const double*, int64_t, double*, int64_t, int, hipStream_t);
template void local_solves_multi<float>(int, int, const int*, const int64_t*, const int*, const int64_t*,
                                        const float*, int, const int64_t*, const unsigned long long*, const double*,
                                        int64_t, double*, int64_t, int, hipStream_t);
template void local_solves<float>(int, int, const int*, const int64_t*, const int*, const int64_t*, const float*, int,
                                  const int64_t*, const unsigned long long*, const double*, double*, bool, int,
                                  hipStream_t, hipEvent_t, hipEvent_t);
template void tile_masks<double>(int, const int64_t*, const int64_t*, const double*, int, const int64_t*,
                                 unsigned long long*, unsigned long long*, hipStream_t);
template void tile_masks<float>(int, const int64_t*, const int64_t*, const float*, int, const int64_t*,
                                unsigned long long*, unsigned long long*, hipStream_t);
template void restrict_phi<double>(int, const int64_t*, const int*, const int64_t*, const int*, const int*,
                                   const int64_t*, const int*, const int64_t*, const double*, const double*, double*,
                                   hipStream_t);
template void restrict_phi<float>(int, const int64_t*, const int*, const int64_t*, const int*, const int*,
                                  const int64_t*, const int*, const int64_t*, const float*, const double*, double*,
                                  hipStream_t);
template void prolong_add<double>(int, int, int64_t, const int*, const int*, const int64_t*, const int*,
                                  const int64_t*, const int*, const int64_t*, const double*, const double*, double*,
                                  hipStream_t);
template void prolong_add<float>(int, int, int64_t, const int*, const int*, const int64_t*, const int*,
                                 const int64_t*, const int*, const int64_t*, const float*, const double*, double*,
                                 hipStream_t);

}  // namespace gdsw
