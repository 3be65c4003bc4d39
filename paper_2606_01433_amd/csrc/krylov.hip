// Kernels of the FGMRES(m) iteration (section 3): CSR SpMV with K,
// classical Gram-Schmidt with reorthogonalisation (dot blocks and AXPY
// blocks), norms and scaling.  Reductions use a fixed two-pass tree, so the
// results do not depend on scheduling.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace gdsw {

namespace {

constexpr int DOT_BLOCK_ROWS = 512;
constexpr int DOT_MAXC = 32;

// One wavefront per row; lane l sums entries l, l + 64, ... in that order, then
// a fixed butterfly.  Rows of up to 512 entries (every row of a Q2-P1disc
// operator) issue all their index, value and gathered loads before the first FMA.
// Up to S entries per lane with every load issued before the first FMA.
template <int S>
__device__ __forceinline__ double spmv_lane(const CsrDev& K, const double* __restrict__ x, int64_t e0, int64_t e1) {
  int c[S];
  double v[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int64_t e = e0 + 64 * j;
    c[j] = (e < e1) ? ld_stream(K.col + e) : 0;
    v[j] = (e < e1) ? ld_stream(K.val + e) : 0.0;
  }
  double xv[S];
#pragma unroll
  for (int j = 0; j < S; ++j) xv[j] = (e0 + 64 * j < e1) ? x[c[j]] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < S; ++j)
    if (e0 + 64 * j < e1) s += v[j] * xv[j];
  return s;
}

// (K x)[row] by one wavefront (every lane returns the sum).
__device__ __forceinline__ double spmv_row(const CsrDev& K, const double* __restrict__ x, int64_t row, int lane) {
  const int64_t e0 = K.rowptr[row] + lane, e1 = K.rowptr[row + 1];
  const int64_t len = e1 - K.rowptr[row];
  double s = 0.0;
  if (len <= 4 * 64) {
    s = spmv_lane<4>(K, x, e0, e1);
  } else if (len <= 8 * 64) {               // vertex rows of Q2 meshes (up to about 410 entries)
    s = spmv_lane<8>(K, x, e0, e1);
  } else {
    for (int64_t e = e0; e < e1; e += 64) s += ld_stream(K.val + e) * x[ld_stream(K.col + e)];
  }
  return wave_sum(s);
}

__global__ __launch_bounds__(256) void k_spmv(CsrDev K, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= K.n) return;
  const int lane = threadIdx.x & 63;
  const double s = spmv_row(K, x, row, lane);
  if (lane == 0) y[row] = s;
}

// Three rows with one column list (offsets ea, eb, ec; len entries each): the columns are read
// and x gathered once; entries base + lane + 64 j (j < S) are added to each row's sum in the order
// spmv_lane takes them.
template <int S>
__device__ __forceinline__ void spmv_lane3(const CsrDev& K, const double* __restrict__ x, int64_t ea, int64_t eb,
                                           int64_t ec, int len, int base, int lane, double& sa, double& sb,
                                           double& sc) {
  int c[S];
  double va[S], vb[S], vc[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int e = base + lane + 64 * j;
    const bool in = e < len;
    c[j] = in ? ld_stream(K.col + ea + e) : 0;
    va[j] = in ? ld_stream(K.val + ea + e) : 0.0;
    vb[j] = in ? ld_stream(K.val + eb + e) : 0.0;
    vc[j] = in ? ld_stream(K.val + ec + e) : 0.0;
  }
  double xv[S];
#pragma unroll
  for (int j = 0; j < S; ++j) xv[j] = (base + lane + 64 * j < len) ? x[c[j]] : 0.0;
#pragma unroll
  for (int j = 0; j < S; ++j)
    if (base + lane + 64 * j < len) {
      sa += va[j] * xv[j];
      sb += vb[j] * xv[j];
      sc += vc[j] * xv[j];
    }
}

// One wavefront per group of three rows; groups flagged in K.same3 share the column reads and
// the gathers of x, the others are three single rows.  Every y[row] equals k_spmv's bit for bit.
__global__ __launch_bounds__(256) void k_spmv3(CsrDev K, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t r0 = 3 * g;
  if (r0 >= K.n) return;
  const int lane = threadIdx.x & 63;
  if (K.same3[g]) {
    const int64_t ea = K.rowptr[r0], eb = K.rowptr[r0 + 1], ec = K.rowptr[r0 + 2];
    const int len = (int)(eb - ea);
    // 256 entries at a time (vertex rows of Q2 meshes take two), which keeps the wave small enough
    // for eight per SIMD; the summation order is spmv_lane's
    double sa = 0.0, sb = 0.0, sc = 0.0;
    for (int base = 0; base < len; base += 4 * 64) spmv_lane3<4>(K, x, ea, eb, ec, len, base, lane, sa, sb, sc);
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    sc = wave_sum(sc);
    if (lane == 0) {
      y[r0] = sa;
      y[r0 + 1] = sb;
      y[r0 + 2] = sc;
    }
    return;
  }
  for (int q = 0; q < 3 && r0 + q < K.n; ++q) {
    const double s = spmv_row(K, x, r0 + q, lane);
    if (lane == 0) y[r0 + q] = s;
  }
}

// same3[g] for every group of three rows (0 for a last, incomplete group); shared[0] += the
// column entries the shared reads save (2 len per flagged group).
__global__ __launch_bounds__(256) void k_same_pattern3(CsrDev K, unsigned char* __restrict__ same3,
                                                       unsigned long long* __restrict__ saved) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t r0 = 3 * g;
  if (r0 >= K.n) return;
  const int lane = threadIdx.x & 63;
  int ok = 0;
  int64_t len = 0;
  if (r0 + 2 < K.n) {
    const int64_t ea = K.rowptr[r0], eb = K.rowptr[r0 + 1], ec = K.rowptr[r0 + 2], ed = K.rowptr[r0 + 3];
    len = eb - ea;
    if (ec - eb == len && ed - ec == len) {
      ok = 1;
      for (int64_t e = lane; e < len; e += 64) {
        const int c = K.col[ea + e];
        if (K.col[eb + e] != c || K.col[ec + e] != c) ok = 0;
      }
      ok = __all(ok);
    }
  }
  if (lane == 0) {
    same3[g] = (unsigned char)ok;
    if (ok) atomicAdd(saved, (unsigned long long)(2 * len));
  }
}

// partial[b * ncols + c] = sum over this block's rows of V[r, c0 + c] w[r].  Thread t takes rows
// r0 + t and r0 + t + 256, in that order; both rows' loads are issued before the first FMA (one
// memory round trip per thread instead of two).
static_assert(DOT_BLOCK_ROWS == 512, "two rows per thread of a 256-thread block");
__global__ __launch_bounds__(256) void k_multi_dot_partial(int64_t n, int ncols, const double* __restrict__ V,
                                                           int64_t ldv, const double* __restrict__ w,
                                                           double* __restrict__ partial, int self,
                                                           const double* __restrict__ gate) {
  if (gate && !(gate[0] > 0.5)) return;
  __shared__ double red[4][DOT_MAXC];
  const int64_t ra = (int64_t)blockIdx.x * DOT_BLOCK_ROWS + threadIdx.x, rb = ra + 256;
  const bool ha = ra < n, hb = rb < n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nout = ncols + self;
  const double wa = ha ? w[ra] : 0.0, wb = hb ? w[rb] : 0.0;
  for (int c0 = 0; c0 < ncols; c0 += DOT_MAXC) {
    const int nc = min(DOT_MAXC, ncols - c0);
    double va[DOT_MAXC], vb[DOT_MAXC];
#pragma unroll
    for (int c = 0; c < DOT_MAXC; ++c) {
      va[c] = (c < nc && ha) ? ld_stream(V + ra + (int64_t)(c0 + c) * ldv) : 0.0;
      vb[c] = (c < nc && hb) ? ld_stream(V + rb + (int64_t)(c0 + c) * ldv) : 0.0;
    }
    double acc[DOT_MAXC];
#pragma unroll
    for (int c = 0; c < DOT_MAXC; ++c) {
      acc[c] = 0.0;
      if (ha) acc[c] += va[c] * wa;
      if (hb) acc[c] += vb[c] * wb;
    }
#pragma unroll
    for (int c = 0; c < DOT_MAXC; ++c) {
      if (c < nc) {
        const double t = wave_sum(acc[c]);
        if (lane == 0) red[wid][c] = t;
      }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
      const int c = threadIdx.x;
      partial[(int64_t)blockIdx.x * nout + c0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
    __syncthreads();
  }
  if (self) {                        // output column ncols: |w|^2
    double acc = 0.0;
    if (ha) acc += wa * wa;
    if (hb) acc += wb * wb;
    const double t = wave_sum(acc);
    if (lane == 0) red[wid][0] = t;
    __syncthreads();
    if (threadIdx.x == 0)
      partial[(int64_t)blockIdx.x * nout + ncols] = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
  }
}

// One wave per column: lanes stride over the block partials, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_multi_dot_reduce(int nblocks, int ncols, const double* __restrict__ partial,
                                                          double* __restrict__ h, const double* __restrict__ gate) {
  if (gate && !(gate[0] > 0.5)) return;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= ncols) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += partial[(int64_t)b * ncols + c];
  s = wave_sum(s);
  if (lane == 0) h[c] = s;
}

// Classical Gram-Schmidt passes over V[:, :ncols] (ncols <= GS_MAXC), each
// reading V once; block partials go to partial[block * nout + c] in a fixed
// order and are summed by k_multi_dot_reduce.  All three are skipped when gate
// is given and not set.
constexpr int GS_MAXC = 250;
constexpr int GS_DOT_ROWS = 2048;   // rows per block of k_gs_dot
constexpr int GS_DOT_COLS = 128;    // columns per block of k_gs_dot (32 per wavefront)
constexpr int GS_ROWS = 64;         // rows per LDS chunk of k_gs_update_dot
constexpr int GS_BLOCKS = 2048;

// Dots of w with the columns, and |w|^2 (output ncols, from the first column
// group): block (x, y) takes rows [x GS_DOT_ROWS, ...) and columns y GS_DOT_COLS
// + wave + 4 i (i < 32), lane = row, accumulating in registers over its rows.
__global__ __launch_bounds__(256) void k_gs_dot(int64_t n, int ncols, const double* __restrict__ V, int64_t ldv,
                                                const double* __restrict__ w, double* __restrict__ partial,
                                                const double* __restrict__ gate) {
  if (gate && !(gate[0] > 0.5)) return;
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int cbase = blockIdx.y * GS_DOT_COLS + wid;
  const int64_t r0 = (int64_t)blockIdx.x * GS_DOT_ROWS;
  const int64_t r1 = min(n, r0 + GS_DOT_ROWS);
  const int nout = ncols + 1;
  double acc[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) acc[i] = 0.0;
  double nacc = 0.0;
  for (int64_t row = r0 + lane; row < r1; row += 64) {
    const double wr = w[row];
    double v[32];
    int64_t o = row + (int64_t)cbase * ldv;   // one running offset (no hoisted per-column addresses)
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      v[i] = cbase + 4 * i < ncols ? ld_stream(V + o) : 0.0;
      o += 4 * ldv;
      asm volatile("" : "+v"(o));
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] += v[i] * wr;
    nacc += wr * wr;
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int c = cbase + 4 * i;
    if (c < ncols) {
      const double t = wave_sum(acc[i]);
      if (lane == 0) partial[(int64_t)blockIdx.x * nout + c] = t;
    }
  }
  if (blockIdx.y == 0) {
    const double t = wave_sum(nacc);
    if (lane == 0) red[wid] = t;
    __syncthreads();
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nout + ncols] = red[0];   // every wave sums the same rows
  }
}

// w -= V h over rows [block GS_DOT_ROWS, ...) (rows strided by 256 per thread,
// columns in order, 32 loads in flight per row), with the block partial of the
// new |w|^2.
__global__ __launch_bounds__(256) void k_gs_update(int64_t n, int ncols, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ h, double* __restrict__ w,
                                                   double* __restrict__ partial, const double* __restrict__ gate) {
  if (gate && !(gate[0] > 0.5)) return;
  __shared__ double hs[GS_MAXC];
  __shared__ double red[4];
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) hs[c] = h[c];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double nacc = 0.0;
  const int64_t r1 = min(n, (int64_t)(blockIdx.x + 1) * GS_DOT_ROWS);
  for (int64_t row = (int64_t)blockIdx.x * GS_DOT_ROWS + threadIdx.x; row < r1; row += 256) {
    double t = 0.0;
    int64_t o = row;
    for (int c0 = 0; c0 < ncols; c0 += 32) {
      double v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        v[i] = c0 + i < ncols ? ld_stream(V + o) : 0.0;
        o += ldv;
        asm volatile("" : "+v"(o));
      }
#pragma unroll
      for (int i = 0; i < 32; ++i)
        if (c0 + i < ncols) t += v[i] * hs[c0 + i];
    }
    const double wn = w[row] - t;
    w[row] = wn;
    nacc += wn * wn;
  }
  const double t = wave_sum(nacc);
  if (lane == 0) red[wid] = t;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// w -= V h, then dots of the new w with the columns and its |w|^2, in chunks of
// GS_ROWS rows (each block a contiguous range of chunks).  The chunk's V values
// are read once: wavefront g = 0..7 takes columns g, g + 8, ... with lane = row
// (coalesced), forms its part of (V h)[row] and stages the values in LDS
// (row-major, odd stride); threads t and t + 256 then sum column t over the
// first and second half of the chunk's rows.  The next chunk's loads are issued
// before the current chunk's dots.
__global__ __launch_bounds__(512) void k_gs_update_dot(int64_t n, int ncols, const double* __restrict__ V,
                                                       int64_t ldv, const double* __restrict__ h,
                                                       double* __restrict__ w, double* __restrict__ partial,
                                                       int64_t chunks_per_block) {
  extern __shared__ double S[];                 // [GS_ROWS][ld]
  __shared__ double hs[GS_MAXC];
  __shared__ double ts[8][GS_ROWS];
  __shared__ double wr[GS_ROWS];
  const int ld = ncols | 1;
  const int t = threadIdx.x, g = t >> 6, r = t & 63;
  const int tc = t & 255, th = t >> 8;          // dot phase: column tc, rows th * 32 ...
  for (int c = t; c < ncols; c += 512) hs[c] = h[c];
  double acc = 0.0, nacc = 0.0;
  const int64_t nchunks = (n + GS_ROWS - 1) / GS_ROWS;
  const int64_t k0 = (int64_t)blockIdx.x * chunks_per_block;
  const int64_t k1 = min(nchunks, k0 + chunks_per_block);
  double v[32];
  auto load = [&](int64_t k) {
    const int64_t row = k * GS_ROWS + r;
    const bool in = k < k1 && row < n;
    int64_t o = row + (int64_t)g * ldv;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      v[u] = (in && g + 8 * u < ncols) ? ld_stream(V + o) : 0.0;
      o += 8 * ldv;
      asm volatile("" : "+v"(o));
    }
  };
  load(k0);
  __syncthreads();   // hs
  for (int64_t k = k0; k < k1; ++k) {
    const int64_t row = k * GS_ROWS + r;
    const bool in = row < n;
    const double wold = (t < GS_ROWS && in) ? w[row] : 0.0;
    double tv = 0.0;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int c = g + 8 * u;
      if (c < ncols) {
        S[r * ld + c] = v[u];
        tv += v[u] * hs[c];
      }
    }
    ts[g][r] = tv;
    load(k + 1);
    __syncthreads();
    if (t < GS_ROWS) {
      const double vh = ((((((ts[0][r] + ts[1][r]) + ts[2][r]) + ts[3][r]) + ts[4][r]) + ts[5][r]) + ts[6][r]) +
                        ts[7][r];
      double wn = wold - vh;
      if (in) w[row] = wn;
      else wn = 0.0;
      nacc += wn * wn;
      wr[r] = wn;
    }
    __syncthreads();
    if (tc < ncols) {
      double d = 0.0;
      const int q0 = th * (GS_ROWS / 2);
#pragma unroll 8
      for (int q = q0; q < q0 + GS_ROWS / 2; ++q) d += S[q * ld + tc] * wr[q];
      acc += d;
    }
    __syncthreads();
  }
  const int nout = ncols + 1;
  double* red = S;                              // [2][ncols], S is free after the last chunk
  if (tc < ncols) red[th * ncols + tc] = acc;
  if (t < 64) {
    const double sn = wave_sum(nacc);
    if (t == 0) partial[(int64_t)blockIdx.x * nout + ncols] = sn;
  }
  __syncthreads();
  if (t < ncols) partial[(int64_t)blockIdx.x * nout + t] = red[t] + red[ncols + t];
}

// Reorthogonalisation test of Daniel, Gragg, Kaufman and Stewart (1976): a
// second Gram-Schmidt pass is needed when the first one removed more than half
// of |w|^2 (|w'|^2 < |w|^2 / 2).  Sets gate; without a second pass the second
// coefficients are zero and |w'|^2 is the final norm.
__global__ void k_gs_decide(int ncols, const double* __restrict__ wn_before, const double* __restrict__ wn_after,
                            double* __restrict__ gate, double* __restrict__ h2, double* __restrict__ nr) {
  const double before = wn_before[0], after = wn_after[0];
  const bool again = after < 0.5 * before;
  for (int c = threadIdx.x; c < ncols; c += blockDim.x)
    if (!again) h2[c] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    gate[0] = again ? 1.0 : 0.0;
    if (!again) nr[0] = after;
  }
}

__global__ __launch_bounds__(256) void k_multi_axpy(int64_t n, int ncols, const double* __restrict__ V, int64_t ldv,
                                                    const double* __restrict__ h, double* __restrict__ w) {
  __shared__ double hs[256];
  for (int c = threadIdx.x; c < ncols && c < 256; c += blockDim.x) hs[c] = h[c];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int c = 0; c < ncols; ++c) acc += ld_stream(V + r + (int64_t)c * ldv) * hs[c];
  w[r] -= acc;
}

__global__ void k_scale_inv_norm(int64_t n, const double* __restrict__ x, const double* __restrict__ nrm2,
                                 double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double nr = sqrt(nrm2[0]);
  y[r] = (nr > 0.0) ? x[r] / nr : 0.0;
}

__global__ void k_residual_from(int64_t n, const double* __restrict__ b, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = b[r] - y[r];
}

// y = a x + b y (y not read when b == 0).
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = (b == 0.0) ? a * x[r] : a * x[r] + b * y[r];
}

}  // namespace

void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, a, x, b, y);
  GDSW_LAUNCH_CHECK();
}

void spmv(const CsrDev& K, const double* x, double* y, hipStream_t s) {
  if (K.same3) {
    hipLaunchKernelGGL(k_spmv3, dim3(blocks_for((K.n + 2) / 3, 4)), dim3(256), 0, s, K, x, y);
  } else {
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(K.n, 4)), dim3(256), 0, s, K, x, y);
  }
  GDSW_LAUNCH_CHECK();
}

void spmv_groups3(const CsrDev& K, unsigned char* same3, unsigned long long* saved, hipStream_t s) {
  hipLaunchKernelGGL(k_same_pattern3, dim3(blocks_for((K.n + 2) / 3, 4)), dim3(256), 0, s, K, same3, saved);
  GDSW_LAUNCH_CHECK();
}

int multi_dot_blocks(int64_t n) { return (int)blocks_for(n, DOT_BLOCK_ROWS); }

void multi_dot(int64_t n, int ncols, const double* V, int64_t ldv, const double* w, double* partial, double* h,
               hipStream_t s) {
  const int nb = multi_dot_blocks(n);
  hipLaunchKernelGGL(k_multi_dot_partial, dim3(nb), dim3(256), 0, s, n, ncols, V, ldv, w, partial, 0,
                     (const double*)nullptr);
  GDSW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_multi_dot_reduce, dim3(blocks_for(ncols, 4)), dim3(256), 0, s, nb, ncols, partial, h,
                     (const double*)nullptr);
  GDSW_LAUNCH_CHECK();
}

void multi_axpy(int64_t n, int ncols, const double* V, int64_t ldv, const double* h, double* w, hipStream_t s) {
  if (ncols > 256) throw Error(-1, "multi_axpy: more than 256 columns");
  hipLaunchKernelGGL(k_multi_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, ncols, V, ldv, h, w);
  GDSW_LAUNCH_CHECK();
}

void gram_schmidt(int64_t n, int ncols, const double* V, int64_t ldv, double* w, double* partial, double* h1,
                  double* h2, double* nr, double* gate, hipStream_t s) {
  if (ncols > GS_MAXC) throw Error(-1, "gram_schmidt: more than 250 columns");
  if (n <= 0 || ncols <= 0) throw Error(-1, "gram_schmidt: empty basis");
  // block counts; each pass writes at most multi_dot_blocks(n) * (ncols + 1) partials
  const int nb_dot = (int)blocks_for(n, GS_DOT_ROWS);
  const int nb_upd = nb_dot;
  const int64_t nchunks = (n + GS_ROWS - 1) / GS_ROWS;
  const int nb_ud = (int)std::min<int64_t>({(int64_t)GS_BLOCKS, nchunks, (int64_t)multi_dot_blocks(n)});
  const int64_t cpb = (nchunks + nb_ud - 1) / nb_ud;
  const size_t lds = (size_t)GS_ROWS * (ncols | 1) * sizeof(double);
  const double* none = nullptr;
  auto reduce = [&](int nb, int count, double* out, const double* g) {
    hipLaunchKernelGGL(k_multi_dot_reduce, dim3(blocks_for(count, 4)), dim3(256), 0, s, nb, count, partial, out, g);
    GDSW_LAUNCH_CHECK();
  };
  // h1 = V^T w and |w|^2 (h1[ncols])
  hipLaunchKernelGGL(k_gs_dot, dim3(nb_dot, (unsigned)blocks_for(ncols, GS_DOT_COLS)), dim3(256), 0, s, n, ncols, V,
                     ldv, w, partial, none);
  GDSW_LAUNCH_CHECK();
  reduce(nb_dot, ncols + 1, h1, none);
  // w -= V h1, with the second coefficients V^T w (kept if needed) and |w|^2 (h2[ncols]) in the same pass
  hipLaunchKernelGGL(k_gs_update_dot, dim3(nb_ud), dim3(512), lds, s, n, ncols, V, ldv, h1, w, partial, cpb);
  GDSW_LAUNCH_CHECK();
  reduce(nb_ud, ncols + 1, h2, none);
  hipLaunchKernelGGL(k_gs_decide, dim3(1), dim3(256), 0, s, ncols, h1 + ncols, h2 + ncols, gate, h2, nr);
  GDSW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gs_update, dim3(nb_upd), dim3(256), 0, s, n, ncols, V, ldv, h2, w, partial, gate);
  GDSW_LAUNCH_CHECK();
  reduce(nb_upd, 1, nr, gate);
}

void scale_by_inv_norm(int64_t n, const double* x, const double* nrm2, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inv_norm, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, nrm2, y);
  GDSW_LAUNCH_CHECK();
}

void residual_from(int64_t n, const double* b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_from, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, b, y);
  GDSW_LAUNCH_CHECK();
}

}  // namespace gdsw
