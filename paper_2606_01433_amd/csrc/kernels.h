// Host-callable launchers of the HIP kernels (all enqueue on the given stream).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace gdsw {

constexpr int LU_NB = 32;   // LU panel width

// A batch of dense column-major square matrices with per-matrix order (ld = order).
struct LuBatch {
  int count = 0;
  int max_n = 0;
  const int64_t* off = nullptr;    // element offset of matrix i
  const int* dim = nullptr;        // order of matrix i
  int* piv = nullptr;              // pivots, matrix i at poff[i]
  const int64_t* poff = nullptr;
  int* info = nullptr;             // first zero pivot (1-based) or 0
  // Columns stored with their length padded to a multiple of `pad` rows
  // (leading dimension lead_dim(order, pad); 0 or 1: ld = order).
  int pad = 0;
  // Optional compact update grids (see LuTiles): per outer step s, prefix sums
  // over the matrices of their 64 x 64 update tiles (device, [steps][count+1]),
  // and the per-step totals (host).  Without them every matrix gets the tiles
  // of the largest one.
  const int64_t* tiles_outer = nullptr;
  const int64_t* tiles_inner = nullptr;
  const int64_t* total_outer = nullptr;
  const int64_t* total_inner = nullptr;
  // Optional device scratch of R * (sum of orders) elements of the batch's type
  // (matrix i at R * poff[i]; R = 64, or 128 when wide): each outer step's U12
  // rows are also written there row-major, so the trailing update reads them with
  // coalesced loads.
  void* ut = nullptr;
  // With ut (R = 128): pairs of 64-column steps share one rank-128 trailing update.
  bool wide = false;
  // Single-matrix batches (count == 1) only: device scratch of
  // lu_tall_scratch_bytes(order, sizeof(T)) bytes.  Panels taller than one
  // workgroup's registers are then factored by many workgroups (one launch per
  // column) instead of by one.
  void* tall_scratch = nullptr;
  // FP64 panels of 769..2048 rows: 0 = two half-width (16-column) register panels, 1 = one
  // full-width panel whenever it fits the registers (an autotuner choice; same pivots and results).
  int full_panels = 0;
  // Size classes for the register panels (an autotuner choice): order = matrix ids by
  // decreasing order (device), order_dims = their orders in that order (host).
  int panel_classes = 0;
  const int* order = nullptr;
  const int* order_dims = nullptr;
  // Optional device scratch of 2 * count words (wide steps only): before each rank-128 trailing
  // update, which 64-row tiles of L21 and 64-column tiles of U12 hold a nonzero; the update skips
  // the C tiles whose product is an exact zero (same result).
  unsigned long long* step_masks = nullptr;
};
size_t lu_tall_scratch_bytes(int n, int value_bytes);
// X = A^{-1} (column-major) of a single LU-factored FP64 matrix (b.count == 1, b.off
// and b.dim its device offset 0 and order n, perm its row permutation) by blocked
// forward and backward sweeps on P I; scratch: 2n + 64 ints of device memory.
void lu_inverse_blocked(const LuBatch& b, const double* LU, const int* perm, double* X, int* scratch, int n,
                        hipStream_t s);

// Host-built update tile tables of a batch with orders dims[0..count).
struct LuTiles {
  std::vector<int64_t> outer, inner;               // [steps][count+1] prefix sums
  std::vector<int64_t> total_outer, total_inner;   // [steps]
  void build(const int* dims, int count);
};

template <typename T> void lu_batched(const LuBatch& b, T* A, hipStream_t s);
template <typename T>
void lu_solve_batched(const LuBatch& b, const T* A, T* X, const int64_t* xoff, const int* nrhs, int max_rhs,
                      hipStream_t s);
void lu_build_perm(const LuBatch& b, int* perm, hipStream_t s);
// A^{-1} of one LU-factored matrix of order n <= 4096 from its factors and row
// permutation (perm[r] = original row at position r), stored by rows:
// out[c + r n] = (A^{-1})[r][c].  Returns false (nothing launched) for larger n.
bool lu_inverse_transposed(const double* LU, const int* perm, double* out, int n, hipStream_t s);

// ---- setup ----------------------------------------------------------------
struct CsrDev {
  int64_t n = 0;
  int64_t nnz = 0;
  const int64_t* rowptr = nullptr;
  const int* col = nullptr;
  const double* val = nullptr;
  // optional: same3[g] = 1 when rows 3g, 3g+1, 3g+2 have identical column lists (the three velocity
  // components of a node); the SpMV then reads those columns and gathers x once for the three rows
  const unsigned char* same3 = nullptr;
};

// Dense local blocks A_i = K[D_i, D_i] (blocks pre-zeroed); one workgroup per
// part in the given order, D_i staged in LDS (max_n = largest order).
template <typename T>
void extract_blocks(const CsrDev& K, int nparts, int max_n, const int* order, const int64_t* dom_ptr, const int* dom,
                    const int64_t* blk_off, T* blocks, int pad, hipStream_t s);
// Interior blocks K[I_i, I_i] and right-hand sides -K[I_i, Gamma] Phi_Gamma (both pre-zeroed).
template <typename T>
void extract_interior(const CsrDev& K, int nparts, int64_t total_rows, const int64_t* int_ptr, const int* inter,
                      const int* dof_ipart, const int* dof_irow, const int* dof_gcol, const int64_t* pc_ptr,
                      const int* pcols, const int64_t* aii_off, T* aii, const int64_t* rhs_off, double* rhs,
                      int* bad, hipStream_t s);
// gidx[k] = D_i[perm_i[a]] for the pivoted gather of the local solves.
void make_gather_index(int nparts, int64_t total, const int64_t* dom_ptr, const int* dom, const int* perm,
                       int* gidx, hipStream_t s);
// Galerkin pieces of part i: W = K[I_i, :] Phi (|I_i| x m_i), V = K[Z_i, I_i] Phi_I (|Z_i| x m_i),
// both stored by rows (row length m_i).
// phit: scratch of the size of phi; it receives Phi_I by rows (part i at phi_off[i], row length m_i),
// which the two products read.
template <typename T>
void galerkin_wv(const CsrDev& K, int nparts, int64_t total_irows, int64_t total_zrows, const int64_t* int_ptr,
                 const int* inter, const int* dof_ipart, const int* dof_irow, const int* dof_gcol,
                 const int64_t* pc_ptr, const int* pcols, const int64_t* phi_off, const T* phi, T* phit,
                 const int64_t* z_ptr, const int* z_dof, const int64_t* v_off, double* W, double* V,
                 int* bad, hipStream_t s);
// C_i = Phi_I^T W + (V rows summed into their columns), m_i x m_i, stored by rows.
template <typename T>
void galerkin_local(int nparts, int64_t total_crows, const int64_t* int_ptr, const int64_t* pc_ptr,
                    const int64_t* phi_off, const T* phi, const double* W, const int64_t* z_ptr, const int* z_lc,
                    const int64_t* v_off, const double* V, const int64_t* c_off, double* C, hipStream_t s);
// A_0 values: interface-interface couplings of K, then every part's C_i in ascending part order.
// The kernels taking `bad` set it to 1 if K couples dofs that share no element of the level
// (the Galerkin decomposition then does not apply; setup reports GDSW_EINVAL).
void galerkin_assemble(const CsrDev& K, const int64_t* col_ptr, const int* col_dofs, const int* dof_gcol,
                       const int64_t* cp_ptr, const int* cp_part, const int* cp_lc, const int64_t* pc_ptr,
                       const int* pcols, const int64_t* c_off, const double* C, const int64_t* a0_rowptr, const int* a0_col,
                       double* a0_val, int n_coarse, int max_row, int* bad, hipStream_t s);
// Dense column-major copy of a CSR matrix (pre-zeroed).
void csr_to_dense(const CsrDev& K, double* D, hipStream_t s);
template <typename T> void set_identity(T* X, int n, hipStream_t s);
template <typename S, typename D> void convert(const S* in, D* out, int64_t n, hipStream_t s);

// ---- apply ----------------------------------------------------------------
// w[k] = local solutions: per part, gather r at gidx, forward/backward TRSV with the LU in place.
// order: part ids, largest block first (the visiting order of the workgroups);
// waves: wavefronts per matrix (2, 4 or 8).  moff/tmask: the nonzero-tile masks from tile_masks;
// the substitution reads only those tiles (and the diagonal ones).
template <typename T>
void local_solves(int nparts, int max_n, const int* order, const int64_t* dom_ptr, const int* gidx,
                  const int64_t* blk_off, const T* blocks, int pad, const int64_t* moff,
                  const unsigned long long* tmask, const double* r, double* w, bool first_level, int waves,
                  hipStream_t s, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Nonzero 64 x 64 tiles of the factored blocks: with nt tiles per side and nw = ceil(nt / 64),
// bit q % 64 of tmask[moff[i] + p nw + q / 64] marks row tile q of column tile p (q != p);
// tmask zeroed beforehand.  kept[0] += the factor elements the masked substitution reads.
template <typename T>
void tile_masks(int nparts, const int64_t* dom_ptr, const int64_t* blk_off, const T* blocks, int pad,
                const int64_t* moff, unsigned long long* tmask, unsigned long long* kept, hipStream_t s);
// The local solves of k right-hand sides (R[s * ldr + g], s < k) into W[s * ldw + position], in chunks
// of local_solves_multi_chunk(max_n, sizeof(T)) right-hand sides per pass over the factors; each column
// agrees with local_solves' result for that right-hand side to rounding (panel updates on MFMA).
template <typename T>
void local_solves_multi(int nparts, int max_n, const int* order, const int64_t* dom_ptr, const int* gidx,
                        const int64_t* blk_off, const T* blocks, int pad, const int64_t* moff,
                        const unsigned long long* tmask, const double* R, int64_t ldr, double* W, int64_t ldw, int k,
                        hipStream_t s);
int local_solves_multi_chunk(int max_n, int value_bytes);
// z[g] = 0.0 + sum_k w[pos[k]] over sc_ptr[g]..sc_ptr[g+1]; with sc_ptr == nullptr, z[g] = 0.0 + w[pos[g]]
void scatter_sum(int64_t n, const int64_t* sc_ptr, const int* sc_pos, const double* w, double* z, hipStream_t s);
// rc = Phi^T r
template <typename T>
void restrict_phi(int n_coarse, const int64_t* col_ptr, const int* col_dofs, const int64_t* cp_ptr,
                  const int* cp_part, const int* cp_lc, const int64_t* int_ptr, const int* inter,
                  const int64_t* phi_off, const T* phi, const double* r, double* rc, hipStream_t s);
// z += Phi y: interface dofs (gdofs, n_gamma of them) take y at their column; interior dofs of
// part i take Phi_I y restricted to the part's columns (max_m = largest column count).
template <typename T>
void prolong_add(int nparts, int max_m, int64_t n_gamma, const int* gdofs, const int* dof_gcol,
                 const int64_t* int_ptr, const int* inter, const int64_t* pc_ptr, const int* pcols,
                 const int64_t* phi_off, const T* phi, const double* y, double* z, hipStream_t s);
// AT = A^T for a dense n x n column-major matrix.
void transpose_square(int n, const double* A, double* AT, hipStream_t s);
// y = Ainv x given AT = Ainv^T (rows of Ainv contiguous); one wave per row, deterministic.
void dense_gemv_rows(int n, const double* AT, const double* x, double* y, hipStream_t s);

// ---- Krylov ---------------------------------------------------------------
void spmv(const CsrDev& K, const double* x, double* y, hipStream_t s);
// K.same3 flags for every group of three rows; *saved += column entries the shared reads save
void spmv_groups3(const CsrDev& K, unsigned char* same3, unsigned long long* saved, hipStream_t s);
// h[c] = V[:, c] . w for c < ncols (V column-major, ld n); partial has blocks*ncols doubles.
void multi_dot(int64_t n, int ncols, const double* V, int64_t ldv, const double* w, double* partial, double* h,
               hipStream_t s);
int multi_dot_blocks(int64_t n);
// Classical Gram-Schmidt of w against V[:, 0..ncols) (ncols <= 250) with a second pass only where
// the test of Daniel, Gragg, Kaufman and Stewart asks for it: h1 = first coefficients (h1[ncols]
// = |w|^2 before), h2 = second coefficients (zero without a second pass), nr[0] = |w|^2 after,
// gate[0] = 1 if the second pass ran.  h1, h2 hold ncols + 1 doubles; partial
// multi_dot_blocks(n) * (ncols + 1).
void gram_schmidt(int64_t n, int ncols, const double* V, int64_t ldv, double* w, double* partial, double* h1,
                  double* h2, double* nr, double* gate, hipStream_t s);
// w -= V[:, 0..ncols) h
void multi_axpy(int64_t n, int ncols, const double* V, int64_t ldv, const double* h, double* w, hipStream_t s);
// y = alpha * x   (alpha read from device: 1 / sqrt(*nrm2))
void scale_by_inv_norm(int64_t n, const double* x, const double* nrm2, double* y, hipStream_t s);
// y = b - y
void residual_from(int64_t n, const double* b, double* y, hipStream_t s);
// y = a x + b y (y is not read when b == 0)
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);

}  // namespace gdsw
