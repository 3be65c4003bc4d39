// Kernels of the FGMRES(m) iteration (section 3): CSR SpMV with K,
// classical Gram-Schmidt with reorthogonalisation (dot blocks and AXPY
// blocks), norms and scaling.  Reductions use a fixed two-pass tree, so the
// results do not depend on scheduling.
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
    c[j] = (e < e1) ? K.col[e] : 0;
    v[j] = (e < e1) ? K.val[e] : 0.0;
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

__global__ __launch_bounds__(256) void k_spmv(CsrDev K, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= K.n) return;
  const int lane = threadIdx.x & 63;
  const int64_t e0 = K.rowptr[row] + lane, e1 = K.rowptr[row + 1];
  const int64_t len = e1 - K.rowptr[row];
  double s = 0.0;
  if (len <= 4 * 64) {
    s = spmv_lane<4>(K, x, e0, e1);
  } else if (len <= 8 * 64) {               // vertex rows of Q2 meshes (up to about 410 entries)
    s = spmv_lane<8>(K, x, e0, e1);
  } else {
    for (int64_t e = e0; e < e1; e += 64) s += K.val[e] * x[K.col[e]];
  }
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// partial[b * ncols + c] = sum over this block's rows of V[r, c0 + c] w[r].  Thread t takes rows
// r0 + t and r0 + t + 256, in that order; both rows' loads are issued before the first FMA (one
// memory round trip per thread instead of two).
static_assert(DOT_BLOCK_ROWS == 512, "two rows per thread of a 256-thread block");
__global__ __launch_bounds__(256) void k_multi_dot_partial(int64_t n, int ncols, const double* __restrict__ V,
                                                           int64_t ldv, const double* __restrict__ w,
                                                           double* __restrict__ partial) {
  __shared__ double red[4][DOT_MAXC];
  const int64_t ra = (int64_t)blockIdx.x * DOT_BLOCK_ROWS + threadIdx.x, rb = ra + 256;
  const bool ha = ra < n, hb = rb < n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncols; c0 += DOT_MAXC) {
    const int nc = min(DOT_MAXC, ncols - c0);
    const double wa = ha ? w[ra] : 0.0, wb = hb ? w[rb] : 0.0;
    double va[DOT_MAXC], vb[DOT_MAXC];
#pragma unroll
    for (int c = 0; c < DOT_MAXC; ++c) {
      va[c] = (c < nc && ha) ? V[ra + (int64_t)(c0 + c) * ldv] : 0.0;
      vb[c] = (c < nc && hb) ? V[rb + (int64_t)(c0 + c) * ldv] : 0.0;
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
      partial[(int64_t)blockIdx.x * ncols + c0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
    __syncthreads();
  }
}

// One wave per column: lanes stride over the block partials, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_multi_dot_reduce(int nblocks, int ncols, const double* __restrict__ partial,
                                                          double* __restrict__ h) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= ncols) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += partial[(int64_t)b * ncols + c];
  s = wave_sum(s);
  if (lane == 0) h[c] = s;
}

// Fused pass of classical Gram-Schmidt: w -= V[:, :ncols] h, then per-block
// partial dots of the updated w with V's columns (norm = 0) or with itself
// (norm = 1).  Same rows per thread, load order and reduction tree as
// k_multi_dot_partial.
__global__ __launch_bounds__(256) void k_axpy_dot_partial(int64_t n, int ncols, const double* __restrict__ V,
                                                          int64_t ldv, const double* __restrict__ h,
                                                          double* __restrict__ w, double* __restrict__ partial,
                                                          int norm) {
  __shared__ double hs[DOT_MAXC];
  __shared__ double red[4][DOT_MAXC];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x < ncols) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  const int64_t ra = (int64_t)blockIdx.x * DOT_BLOCK_ROWS + threadIdx.x, rb = ra + 256;
  const bool ha = ra < n, hb = rb < n;
  const int nout = norm ? 1 : ncols;
  double va[DOT_MAXC], vb[DOT_MAXC];
#pragma unroll
  for (int c = 0; c < DOT_MAXC; ++c) {
    va[c] = (c < ncols && ha) ? V[ra + (int64_t)c * ldv] : 0.0;
    vb[c] = (c < ncols && hb) ? V[rb + (int64_t)c * ldv] : 0.0;
  }
  const double wa0 = ha ? w[ra] : 0.0, wb0 = hb ? w[rb] : 0.0;
  double acc[DOT_MAXC];
#pragma unroll
  for (int c = 0; c < DOT_MAXC; ++c) acc[c] = 0.0;
  auto row = [&](const double* v, double w0, int64_t r) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < DOT_MAXC; ++c) t += v[c] * hs[min(c, ncols - 1)] * (c < ncols ? 1.0 : 0.0);
    const double wr = w0 - t;
    w[r] = wr;
    if (norm) {
      acc[0] += wr * wr;
    } else {
#pragma unroll
      for (int c = 0; c < DOT_MAXC; ++c)
        if (c < ncols) acc[c] += v[c] * wr;
    }
  };
  if (ha) row(va, wa0, ra);
  if (hb) row(vb, wb0, rb);
#pragma unroll
  for (int c = 0; c < DOT_MAXC; ++c) {
    if (c < nout) {
      const double t = wave_sum(acc[c]);
      if (lane == 0) red[wid][c] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x < nout) {
    const int c = threadIdx.x;
    partial[(int64_t)blockIdx.x * nout + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
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
  for (int c = 0; c < ncols; ++c) acc += V[r + (int64_t)c * ldv] * hs[c];
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
  hipLaunchKernelGGL(k_spmv, dim3(blocks_for(K.n, 4)), dim3(256), 0, s, K, x, y);
  GDSW_LAUNCH_CHECK();
}

int multi_dot_blocks(int64_t n) { return (int)blocks_for(n, DOT_BLOCK_ROWS); }

void multi_dot(int64_t n, int ncols, const double* V, int64_t ldv, const double* w, double* partial, double* h,
               hipStream_t s) {
  const int nb = multi_dot_blocks(n);
  hipLaunchKernelGGL(k_multi_dot_partial, dim3(nb), dim3(256), 0, s, n, ncols, V, ldv, w, partial);
  GDSW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_multi_dot_reduce, dim3(blocks_for(ncols, 4)), dim3(256), 0, s, nb, ncols, partial, h);
  GDSW_LAUNCH_CHECK();
}

int fused_gs_max_cols() { return DOT_MAXC; }

void axpy_dot(int64_t n, int ncols, const double* V, int64_t ldv, const double* h, double* w, double* partial,
              double* out, bool norm, hipStream_t s) {
  if (ncols > DOT_MAXC) throw Error(-1, "axpy_dot: too many columns");
  const int nb = multi_dot_blocks(n);
  hipLaunchKernelGGL(k_axpy_dot_partial, dim3(nb), dim3(256), 0, s, n, ncols, V, ldv, h, w, partial, norm ? 1 : 0);
  GDSW_LAUNCH_CHECK();
  const int nout = norm ? 1 : ncols;
  hipLaunchKernelGGL(k_multi_dot_reduce, dim3(blocks_for(nout, 4)), dim3(256), 0, s, nb, nout, partial, out);
  GDSW_LAUNCH_CHECK();
}

void multi_axpy(int64_t n, int ncols, const double* V, int64_t ldv, const double* h, double* w, hipStream_t s) {
  if (ncols > 256) throw Error(-1, "multi_axpy: more than 256 columns");
  hipLaunchKernelGGL(k_multi_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, ncols, V, ldv, h, w);
  GDSW_LAUNCH_CHECK();
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
