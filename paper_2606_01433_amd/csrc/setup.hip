// Setup kernels: local block extraction (section 2.1, A_i = R_i K R_i^T), the
// interior problems of the GDSW extension (Phi_I = -A_II^{-1} A_{I,Gamma}
// Phi_Gamma) and the Galerkin product A_0 = Phi^T K Phi.
//
// The Galerkin product is evaluated part by part.  Every coupling K[g, h]
// with g or h interior to part i lies inside the closure of part i, so
//   A_0 = sum_{g,h in Gamma} e_col(g) K[g,h] e_col(h)^T
//       + sum_i ( Phi_I,i^T (K Phi)[I_i, :] + (K[Z_i, I_i] Phi_I,i) summed into rows col(Z_i) ),
// where Z_i are the interface dofs of part i's closure.  All sums run in a
// fixed order (no atomics), so the result is reproducible bit for bit.
#include "common.h"
#include "kernels.h"

namespace gdsw {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_extract_blocks(CsrDev K, const int* __restrict__ order,
                                                        const int64_t* __restrict__ dom_ptr,
                                                        const int* __restrict__ dom,
                                                        const int64_t* __restrict__ blk_off, T* __restrict__ blocks,
                                                        int pad) {
  // one workgroup per part (largest first); the part's sorted dof list lives
  // in LDS for the binary searches, one wave per local row
  extern __shared__ int sD[];
  const int i = order[blockIdx.x];
  const int64_t base = dom_ptr[i];
  const int n = (int)(dom_ptr[i + 1] - base);
  for (int a = threadIdx.x; a < n; a += blockDim.x) sD[a] = dom[base + a];
  __syncthreads();
  T* A = blocks + blk_off[i];
  const int ld = lead_dim(n, pad);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int a = wid; a < n; a += nw) {
    const int g = sD[a];
    for (int64_t e = K.rowptr[g] + lane; e < K.rowptr[g + 1]; e += 64) {
      const int h = K.col[e];
      const int b = lower_bound_i32(sD, n, h);
      if (b < n && sD[b] == h) A[a + (int64_t)b * ld] = (T)K.val[e];
    }
  }
}

// Interior block rows and right-hand sides, one wave per interior row: the
// lanes fetch 64 couplings of the row and classify them; interior couplings
// are stored directly, interface couplings are summed into the right-hand
// side in row order (lane c owns coarse column c; R starts at zero).
template <typename T>
__global__ __launch_bounds__(256) void k_extract_interior(CsrDev K, int nparts, int64_t total_rows,
                                                          const int64_t* __restrict__ int_ptr,
                                                          const int* __restrict__ inter,
                                                          const int* __restrict__ dof_ipart,
                                                          const int* __restrict__ dof_irow,
                                                          const int* __restrict__ dof_gcol,
                                                          const int64_t* __restrict__ pc_ptr,
                                                          const int* __restrict__ pcols,
                                                          const int64_t* __restrict__ aii_off, T* __restrict__ aii,
                                                          const int64_t* __restrict__ rhs_off,
                                                          double* __restrict__ rhs, int* __restrict__ bad) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= total_rows) return;
  const int lane = threadIdx.x & 63;
  const int i = segment_of(int_ptr, nparts, row);
  const int64_t base = int_ptr[i];
  const int nI = (int)(int_ptr[i + 1] - base);
  const int a = (int)(row - base);
  const int g = inter[row];
  const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
  const int* pc = pcols + pc_ptr[i];
  T* A = aii + aii_off[i];
  double* R = rhs + rhs_off[i];
  const int64_t e_beg = K.rowptr[g], e_end = K.rowptr[g + 1];
  for (int c0 = 0; c0 < m || c0 == 0; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    for (int64_t e0 = e_beg; e0 < e_end; e0 += 64) {
      const int64_t e = e0 + lane;
      int lc = -1;
      double v = 0.0;
      if (e < e_end) {
        const int h = K.col[e];
        v = K.val[e];
        if (dof_ipart[h] == i) {
          if (c0 == 0) A[a + (int64_t)dof_irow[h] * nI] = (T)v;
        } else {
          const int gc = dof_gcol[h];
          const int p = gc >= 0 ? lower_bound_i32(pc, m, gc) : m;
          if (p < m && pc[p] == gc) lc = p;
          else if (gc >= 0 || dof_ipart[h] >= 0) *bad = 1;   // K couples an interior dof outside its
                                                             // part's closure (an interface dof without
                                                             // a coarse column has Phi = 0: no term)
        }
      }
      const int cnt = (int)min((int64_t)64, e_end - e0);
      for (int l = 0; l < cnt; ++l) {
        const int lcl = lane_value(lc, l);
        if (lcl >= 0 && lcl == c) acc -= lane_value(v, l);
      }
    }
    if (c < m) R[a + (int64_t)c * nI] = acc;
  }
}

__global__ void k_gather_index(int nparts, int64_t total, const int64_t* __restrict__ dom_ptr,
                               const int* __restrict__ dom, const int* __restrict__ perm, int* __restrict__ gidx) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  const int i = segment_of(dom_ptr, nparts, k);
  gidx[k] = dom[dom_ptr[i] + perm[k]];
}

// W[a, c] = sum_h K[g_a, h] Phi[h, c] over the row of interior dof g_a (one wave per row).
// The lanes first fetch 64 couplings of the row and classify them (interior row
// or interface column of this part); the couplings are then applied in row
// order, lane c accumulating column c.
template <typename T>
__global__ __launch_bounds__(256) void k_galerkin_w(CsrDev K, int nparts, int64_t total_rows,
                                                    const int64_t* __restrict__ int_ptr,
                                                    const int* __restrict__ inter, const int* __restrict__ dof_ipart,
                                                    const int* __restrict__ dof_irow,
                                                    const int* __restrict__ dof_gcol,
                                                    const int64_t* __restrict__ pc_ptr, const int* __restrict__ pcols,
                                                    const int64_t* __restrict__ phi_off, const T* __restrict__ phit,
                                                    double* __restrict__ W, int* __restrict__ bad) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= total_rows) return;
  const int lane = threadIdx.x & 63;
  const int i = segment_of(int_ptr, nparts, row);
  const int64_t base = int_ptr[i];
  const int a = (int)(row - base);
  const int g = inter[row];
  const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
  const int* pc = pcols + pc_ptr[i];
  const T* ph = phit + phi_off[i];           // Phi_I of the part by rows
  double* Wp = W + phi_off[i];
  const int64_t e_beg = K.rowptr[g], e_end = K.rowptr[g + 1];
  for (int c0 = 0; c0 < m; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    for (int64_t e0 = e_beg; e0 < e_end; e0 += 64) {
      const int64_t e = e0 + lane;
      int ir = -1, lc = -1;
      double v = 0.0;
      if (e < e_end) {
        const int h = K.col[e];
        v = K.val[e];
        if (dof_ipart[h] == i) {
          ir = dof_irow[h];
        } else {
          const int gc = dof_gcol[h];
          const int p = gc >= 0 ? lower_bound_i32(pc, m, gc) : m;
          if (p < m && pc[p] == gc) lc = p;
          else if (gc >= 0 || dof_ipart[h] >= 0) *bad = 1;   // as in k_extract_interior
        }
      }
      const int cnt = (int)min((int64_t)64, e_end - e0);
      for (int l = 0; l < cnt; ++l) {
        const double vl = lane_value(v, l);
        const int irl = lane_value(ir, l);
        if (irl >= 0) {
          if (c < m) acc += vl * (double)ph[(int64_t)irl * m + c];
        } else if (lane_value(lc, l) == c) {
          acc += vl;
        }
      }
    }
    if (c < m) Wp[(int64_t)a * m + c] = acc;
  }
}

// V[t, c] = sum_{h in I_i} K[z_t, h] Phi_I[h, c] for the interface dofs z_t of part i's closure.
template <typename T>
__global__ __launch_bounds__(256) void k_galerkin_v(CsrDev K, int nparts, int64_t total_rows,
                                                    const int64_t* __restrict__ z_ptr, const int* __restrict__ z_dof,
                                                    const int64_t* __restrict__ int_ptr,
                                                    const int* __restrict__ dof_ipart,
                                                    const int* __restrict__ dof_irow,
                                                    const int64_t* __restrict__ pc_ptr,
                                                    const int64_t* __restrict__ phi_off, const T* __restrict__ phit,
                                                    const int64_t* __restrict__ v_off, double* __restrict__ V) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= total_rows) return;
  const int lane = threadIdx.x & 63;
  const int i = segment_of(z_ptr, nparts, row);
  const int64_t base = z_ptr[i];
  const int t = (int)(row - base);
  const int g = z_dof[row];
  const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
  const T* ph = phit + phi_off[i];           // Phi_I of the part by rows
  double* Vp = V + v_off[i];
  const int64_t e_beg = K.rowptr[g], e_end = K.rowptr[g + 1];
  for (int c0 = 0; c0 < m; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    for (int64_t e0 = e_beg; e0 < e_end; e0 += 64) {
      const int64_t e = e0 + lane;
      int ir = -1;
      double v = 0.0;
      if (e < e_end) {
        const int h = K.col[e];
        if (dof_ipart[h] == i) {
          ir = dof_irow[h];
          v = K.val[e];
        }
      }
      const int cnt = (int)min((int64_t)64, e_end - e0);
      for (int l = 0; l < cnt; ++l) {
        const int irl = lane_value(ir, l);
        if (irl >= 0 && c < m) acc += lane_value(v, l) * (double)ph[(int64_t)irl * m + c];
      }
    }
    if (c < m) Vp[(int64_t)t * m + c] = acc;
  }
}

// Phi_I of part i (|I_i| x m_i, by columns) copied by rows; one workgroup per part.
template <typename T>
__global__ __launch_bounds__(256) void k_phi_rows(const int64_t* __restrict__ int_ptr,
                                                  const int64_t* __restrict__ pc_ptr,
                                                  const int64_t* __restrict__ phi_off, const T* __restrict__ phi,
                                                  T* __restrict__ phit) {
  const int i = blockIdx.x;
  const int nI = (int)(int_ptr[i + 1] - int_ptr[i]);
  const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
  const T* src = phi + phi_off[i];
  T* dst = phit + phi_off[i];
  const int64_t total = (int64_t)nI * m;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int r = (int)(e / m), c = (int)(e - (int64_t)r * m);
    dst[e] = src[r + (int64_t)c * nI];
  }
}

// C_i[r, c] = sum_a Phi_I[a, r] W[a, c] + sum_{t : lc(t) = r} V[t, c]   (one wave per (part, r))
template <typename T>
__global__ __launch_bounds__(256) void k_galerkin_local(int nparts, int64_t total_rows,
                                                        const int64_t* __restrict__ int_ptr,
                                                        const int64_t* __restrict__ pc_ptr,
                                                        const int64_t* __restrict__ phi_off, const T* __restrict__ phi,
                                                        const double* __restrict__ W,
                                                        const int64_t* __restrict__ z_ptr, const int* __restrict__ z_lc,
                                                        const int64_t* __restrict__ v_off,
                                                        const double* __restrict__ V,
                                                        const int64_t* __restrict__ c_off, double* __restrict__ C) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= total_rows) return;
  const int lane = threadIdx.x & 63;
  const int i = segment_of(pc_ptr, nparts, row);
  const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
  const int r = (int)(row - pc_ptr[i]);
  const int nI = (int)(int_ptr[i + 1] - int_ptr[i]);
  const T* ph = phi + phi_off[i] + (int64_t)r * nI;
  const double* Wp = W + phi_off[i];
  const int64_t zb = z_ptr[i];
  const int nZ = (int)(z_ptr[i + 1] - zb);
  const int* zl = z_lc + zb;
  const int t0 = lower_bound_i32(zl, nZ, r);
  const int t1 = lower_bound_i32(zl, nZ, r + 1);
  const double* Vp = V + v_off[i];
  double* Cp = C + c_off[i];
  for (int c0 = 0; c0 < m; c0 += 64) {
    const int c = c0 + lane;
    if (c >= m) break;
    double acc = 0.0;
    for (int a = 0; a < nI; ++a) acc += (double)ph[a] * Wp[(int64_t)a * m + c];
    for (int t = t0; t < t1; ++t) acc += Vp[(int64_t)t * m + c];
    Cp[(int64_t)r * m + c] = acc;
  }
}

// One wave per coarse row c, accumulating in wave-private LDS: the
// interface-interface couplings of K (dof by dof, in row order), then the
// parts' C_i in ascending part order.  Lanes look up 64 contributions at a
// time; the additions are applied in that fixed order through readlane.
__global__ __launch_bounds__(64) void k_galerkin_assemble(CsrDev K, const int64_t* __restrict__ col_ptr,
                                                          const int* __restrict__ col_dofs,
                                                          const int* __restrict__ dof_gcol,
                                                          const int64_t* __restrict__ cp_ptr,
                                                          const int* __restrict__ cp_part,
                                                          const int* __restrict__ cp_lc,
                                                          const int64_t* __restrict__ pc_ptr,
                                                          const int* __restrict__ pcols,
                                                          const int64_t* __restrict__ c_off,
                                                          const double* __restrict__ C,
                                                          const int64_t* __restrict__ a0_rowptr,
                                                          const int* __restrict__ a0_col, double* __restrict__ a0_val,
                                                          int n_coarse, int* __restrict__ bad) {
  extern __shared__ double rv[];
  const int c = blockIdx.x;
  if (c >= n_coarse) return;
  const int lane = threadIdx.x;
  const int64_t rb = a0_rowptr[c];
  const int len = (int)(a0_rowptr[c + 1] - rb);
  const int* rc = a0_col + rb;
  for (int k = lane; k < len; k += 64) rv[k] = 0.0;
  __syncthreads();
  for (int64_t q = col_ptr[c]; q < col_ptr[c + 1]; ++q) {
    const int g = col_dofs[q];
    const int64_t e_beg = K.rowptr[g], e_end = K.rowptr[g + 1];
    for (int64_t e0 = e_beg; e0 < e_end; e0 += 64) {
      const int64_t e = e0 + lane;
      int pos = -1;
      double v = 0.0;
      if (e < e_end) {
        const int gc = dof_gcol[K.col[e]];
        if (gc >= 0) {
          const int p = lower_bound_i32(rc, len, gc);
          if (p < len && rc[p] == gc) {
            pos = p;
            v = K.val[e];
          } else {
            *bad = 1;
          }
        }
      }
      const int cnt = (int)min((int64_t)64, e_end - e0);
      for (int l = 0; l < cnt; ++l) {
        const int pl = lane_value(pos, l);
        const double vl = lane_value(v, l);
        if (pl >= 0 && lane == (pl & 63)) rv[pl] += vl;
      }
    }
  }
  for (int64_t t = cp_ptr[c]; t < cp_ptr[c + 1]; ++t) {
    const int i = cp_part[t];
    const int lc = cp_lc[t];
    const int m = (int)(pc_ptr[i + 1] - pc_ptr[i]);
    const int* pc = pcols + pc_ptr[i];
    const double* Ci = C + c_off[i];
    for (int l0 = 0; l0 < m; l0 += 64) {
      const int l2 = l0 + lane;
      int pos = -1;
      double v = 0.0;
      if (l2 < m) {
        const int p = lower_bound_i32(rc, len, pc[l2]);
        if (p < len && rc[p] == pc[l2]) {
          pos = p;
          v = Ci[(int64_t)lc * m + l2];
        } else {
          *bad = 1;
        }
      }
      // distinct columns of one part land on distinct positions: no ordering conflict
      if (pos >= 0) rv[pos] += v;
    }
  }
  __syncthreads();
  for (int k = lane; k < len; k += 64) a0_val[rb + k] = rv[k];
}

__global__ void k_csr_to_dense(CsrDev K, double* __restrict__ D) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= K.n) return;
  for (int64_t e = K.rowptr[r]; e < K.rowptr[r + 1]; ++e) D[r + (int64_t)K.col[e] * K.n] = K.val[e];
}

template <typename T>
__global__ void k_set_identity(T* X, int n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)n * n) return;
  X[k] = ((k % n) == (k / n)) ? T(1) : T(0);
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ in, D* __restrict__ out, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = (D)in[k];
}

}  // namespace

template <typename T>
void extract_blocks(const CsrDev& K, int nparts, int max_n, const int* order, const int64_t* dom_ptr, const int* dom,
                    const int64_t* blk_off, T* blocks, int pad, hipStream_t s) {
  if (nparts == 0) return;
  if ((size_t)max_n * sizeof(int) > 64 * 1024) throw Error(-1, "extract_blocks: local block too large");
  hipLaunchKernelGGL((k_extract_blocks<T>), dim3(nparts), dim3(256), (size_t)max_n * sizeof(int), s, K, order,
                     dom_ptr, dom, blk_off, blocks, pad);
  GDSW_LAUNCH_CHECK();
}

template <typename T>
void extract_interior(const CsrDev& K, int nparts, int64_t total_rows, const int64_t* int_ptr, const int* inter,
                      const int* dof_ipart, const int* dof_irow, const int* dof_gcol, const int64_t* pc_ptr,
                      const int* pcols, const int64_t* aii_off, T* aii, const int64_t* rhs_off, double* rhs,
                      int* bad, hipStream_t s) {
  if (total_rows == 0) return;
  hipLaunchKernelGGL((k_extract_interior<T>), dim3(blocks_for(total_rows, 4)), dim3(256), 0, s, K, nparts,
                     total_rows, int_ptr, inter, dof_ipart, dof_irow, dof_gcol, pc_ptr, pcols, aii_off, aii, rhs_off,
                     rhs, bad);
  GDSW_LAUNCH_CHECK();
}

void make_gather_index(int nparts, int64_t total, const int64_t* dom_ptr, const int* dom, const int* perm,
                       int* gidx, hipStream_t s) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_gather_index, dim3(blocks_for(total, 256)), dim3(256), 0, s, nparts, total, dom_ptr, dom,
                     perm, gidx);
  GDSW_LAUNCH_CHECK();
}

template <typename T>
void galerkin_wv(const CsrDev& K, int nparts, int64_t total_irows, int64_t total_zrows, const int64_t* int_ptr,
                 const int* inter, const int* dof_ipart, const int* dof_irow, const int* dof_gcol,
                 const int64_t* pc_ptr, const int* pcols, const int64_t* phi_off, const T* phi, T* phit,
                 const int64_t* z_ptr, const int* z_dof, const int64_t* v_off, double* W, double* V,
                 int* bad, hipStream_t s) {
  if (nparts > 0) {
    hipLaunchKernelGGL((k_phi_rows<T>), dim3(nparts), dim3(256), 0, s, int_ptr, pc_ptr, phi_off, phi, phit);
    GDSW_LAUNCH_CHECK();
  }
  if (total_irows > 0) {
    hipLaunchKernelGGL((k_galerkin_w<T>), dim3(blocks_for(total_irows, 4)), dim3(256), 0, s, K, nparts,
                       total_irows, int_ptr, inter, dof_ipart, dof_irow, dof_gcol, pc_ptr, pcols, phi_off, phit, W,
                       bad);
    GDSW_LAUNCH_CHECK();
  }
  if (total_zrows > 0) {
    hipLaunchKernelGGL((k_galerkin_v<T>), dim3(blocks_for(total_zrows, 4)), dim3(256), 0, s, K, nparts,
                       total_zrows, z_ptr, z_dof, int_ptr, dof_ipart, dof_irow, pc_ptr, phi_off, phit, v_off, V);
    GDSW_LAUNCH_CHECK();
  }
}

template <typename T>
void galerkin_local(int nparts, int64_t total_crows, const int64_t* int_ptr, const int64_t* pc_ptr,
                    const int64_t* phi_off, const T* phi, const double* W, const int64_t* z_ptr, const int* z_lc,
                    const int64_t* v_off, const double* V, const int64_t* c_off, double* C, hipStream_t s) {
  if (total_crows == 0) return;
  hipLaunchKernelGGL((k_galerkin_local<T>), dim3(blocks_for(total_crows, 4)), dim3(256), 0, s, nparts, total_crows,
                     int_ptr, pc_ptr, phi_off, phi, W, z_ptr, z_lc, v_off, V, c_off, C);
  GDSW_LAUNCH_CHECK();
}

void galerkin_assemble(const CsrDev& K, const int64_t* col_ptr, const int* col_dofs, const int* dof_gcol,
                       const int64_t* cp_ptr, const int* cp_part, const int* cp_lc, const int64_t* pc_ptr,
                       const int* pcols, const int64_t* c_off, const double* C, const int64_t* a0_rowptr,
                       const int* a0_col, double* a0_val, int n_coarse, int max_row, int* bad, hipStream_t s) {
  if (n_coarse == 0) return;
  if ((size_t)max_row * sizeof(double) > 64 * 1024) throw Error(-1, "coarse row too long for the LDS accumulator");
  hipLaunchKernelGGL(k_galerkin_assemble, dim3(n_coarse), dim3(64), (size_t)max_row * sizeof(double), s, K, col_ptr,
                     col_dofs, dof_gcol, cp_ptr, cp_part, cp_lc, pc_ptr, pcols, c_off, C, a0_rowptr, a0_col, a0_val,
                     n_coarse, bad);
  GDSW_LAUNCH_CHECK();
}

void csr_to_dense(const CsrDev& K, double* D, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_to_dense, dim3(blocks_for(K.n, 128)), dim3(128), 0, s, K, D);
  GDSW_LAUNCH_CHECK();
}

template <typename T>
void set_identity(T* X, int n, hipStream_t s) {
  hipLaunchKernelGGL((k_set_identity<T>), dim3(blocks_for((int64_t)n * n, 256)), dim3(256), 0, s, X, n);
  GDSW_LAUNCH_CHECK();
}

template <typename S, typename D>
void convert(const S* in, D* out, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_convert<S, D>), dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
  GDSW_LAUNCH_CHECK();
}

template void extract_blocks<double>(const CsrDev&, int, int, const int*, const int64_t*, const int*,
                                     const int64_t*, double*, int, hipStream_t);
template void extract_blocks<float>(const CsrDev&, int, int, const int*, const int64_t*, const int*, const int64_t*,
                                    float*, int, hipStream_t);
template void extract_interior<double>(const CsrDev&, int, int64_t, const int64_t*, const int*, const int*,
                                       const int*, const int*, const int64_t*, const int*, const int64_t*, double*,
                                       const int64_t*, double*, int*, hipStream_t);
template void extract_interior<float>(const CsrDev&, int, int64_t, const int64_t*, const int*, const int*,
                                      const int*, const int*, const int64_t*, const int*, const int64_t*, float*,
                                      const int64_t*, double*, int*, hipStream_t);
template void galerkin_wv<double>(const CsrDev&, int, int64_t, int64_t, const int64_t*, const int*, const int*,
                                  const int*, const int*, const int64_t*, const int*, const int64_t*, const double*, double*,
                                  const int64_t*, const int*, const int64_t*, double*, double*, int*, hipStream_t);
template void galerkin_wv<float>(const CsrDev&, int, int64_t, int64_t, const int64_t*, const int*, const int*,
                                 const int*, const int*, const int64_t*, const int*, const int64_t*, const float*, float*,
                                 const int64_t*, const int*, const int64_t*, double*, double*, int*, hipStream_t);
template void galerkin_local<double>(int, int64_t, const int64_t*, const int64_t*, const int64_t*, const double*,
                                     const double*, const int64_t*, const int*, const int64_t*, const double*,
                                     const int64_t*, double*, hipStream_t);
template void galerkin_local<float>(int, int64_t, const int64_t*, const int64_t*, const int64_t*, const float*,
                                    const double*, const int64_t*, const int*, const int64_t*, const double*,
                                    const int64_t*, double*, hipStream_t);
template void set_identity<double>(double*, int, hipStream_t);
template void convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void convert<float, double>(const float*, double*, int64_t, hipStream_t);

}  // namespace gdsw
