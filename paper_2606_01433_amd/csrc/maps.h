// Host-side index maps of one level of the multilevel GDSW hierarchy.
//
// Section 2.1 defines the overlapping subdomains, the interface and its
// entities (vertices, edges, faces), the interior sets and the interface
// part of the coarse basis; section 2.2 recurses on the coarse problem.
// These are pure integer graph computations done once per setup on the host;
// every floating-point step runs in the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <functional>
#include <memory>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

namespace gdsw {

// Allocator whose resize leaves new elements default-initialized (integers are left unset): the
// large index arrays below are sized and then filled in parallel, without a serial zeroing pass.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() noexcept = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <typename T>
using RawVec = std::vector<T, NoInitAlloc<T>>;

// One level: nodes carrying up to three velocity dofs, elements with a node
// list and four pressure slots (mode 0 constant, modes 1..3 linear), parts.
struct LevelMesh {
  int n_dof = 0;
  int n_nodes = 0;
  std::vector<int> node_dof;          // n_nodes*3, -1 = no dof
  int n_elem = 0;
  std::vector<int64_t> en_ptr;        // element -> nodes (CSR)
  RawVec<int> en;
  std::vector<int> elem_pdof;         // n_elem*4, -1 = none
  std::vector<int> elem_part;         // n_elem
  int n_parts = 0;
  std::vector<int64_t> adj_ptr;       // node graph (sorted, no self loops)
  RawVec<int> adj;
  std::vector<int64_t> ne_ptr;        // node -> elements (ascending), when the builder made it
  RawVec<int> ne;
};

struct LevelMaps {
  // S(v): parts of the elements that contain node v (sorted)
  std::vector<int64_t> s_ptr;
  std::vector<int> s;
  std::vector<int> gamma_nodes;       // nodes with a free dof in >= 2 parts
  std::vector<int> node_ent;          // entity of an interface node, else -1
  std::vector<int64_t> ent_ptr;
  std::vector<int> ent_nodes;
  std::vector<int> ent_kind;          // 0 vertex, 1 edge, 2 face
  std::vector<int64_t> es_ptr;        // S(E) per entity
  std::vector<int> es;
  // coarse columns (= dofs of the next level)
  int n_coarse = 0;
  std::vector<int> col_entity;        // entity, or -1-part for a pressure column
  std::vector<int> col_dir;           // 0..2, 3 = pressure
  std::vector<int64_t> col_ptr;       // dofs where Phi_Gamma has a one
  std::vector<int> col_dofs;
  std::vector<int> ent_col;           // n_ent*3, -1 = no column
  std::vector<int> part_col;          // n_parts, -1 = no pressure column
  // overlapping sets D_i and interior sets I_i (sorted dof lists)
  std::vector<int64_t> dom_ptr;
  RawVec<int> dom;
  std::vector<int64_t> int_ptr;
  std::vector<int> inter;
  // per-dof tables
  RawVec<int> owner;                  // owning part (restricted combination)
  RawVec<int> dof_gcol;               // coarse column of an interface dof, else -1
  RawVec<int> dof_ipart;              // part of an interior dof, else -1
  RawVec<int> dof_irow;               // row of an interior dof inside I_i
  // per part: coarse columns touching the part (sorted)
  std::vector<int64_t> pc_ptr;
  std::vector<int> pcols;
  // per coarse column: parts that hold it and its index in their column list
  std::vector<int64_t> cp_ptr;
  std::vector<int> cp_part;
  std::vector<int> cp_lc;
  // per part: interface dofs of its closure, sorted by (local column, dof)
  std::vector<int64_t> z_ptr;
  std::vector<int> z_dof;
  std::vector<int> z_lc;
};

// Validates the caller's level-1 description; returns "" or an error text.
std::string build_level1_mesh(int64_t n, int n_nodes, const int* node_dof, int n_elem,
                              const int* elem_node, const int* elem_pdof, const int* elem_part,
                              int n_parts, LevelMesh& out);

// S(v), the owning part of every dof and the overlapping sets D_i (dom_ptr /
// dom) only: everything the local factorizations need.
void build_domains(const LevelMesh& mesh, int delta, LevelMaps& m);

// All maps of the level; reuses D_i (and S, owner) when build_domains ran on m.
// linear_interior: the linear pressure modes (1..3) of a part's elements are
// interior dofs of the part (a saddle-point extension); false: they are
// interface dofs that no coarse column touches (a velocity-only extension).
void build_maps(const LevelMesh& mesh, int delta, LevelMaps& m, bool linear_interior = true);

// Mesh of the next level: entities become nodes, parts become elements.
std::string build_next_mesh(const LevelMesh& mesh, const LevelMaps& m, const int* parent,
                            int n_parts_next, LevelMesh& out);

// Sparsity of A_0 = Phi^T K Phi: row c holds the union of the column lists
// of the parts that hold column c.
void coarse_pattern(const LevelMaps& m, std::vector<int64_t>& rowptr, std::vector<int>& col);

// work(t) for t in [0, nthreads) on the process-wide host worker threads (the
// caller runs t = 0), or on threads created for this call while another caller
// holds them.  nthreads is capped by the host thread count.
void host_parallel(int nthreads, const std::function<void(int)>& work);
int host_thread_count();

// Combination lists of the local solutions: additive lists every position of
// dof g over all domains (sc_ptr / sc_pos, ascending position); restricted
// lists only the position inside the owner's domain (sc_pos[g], sc_ptr left
// empty).  Returns "" or an error text.
std::string scatter_lists(const LevelMaps& m, int64_t n, bool additive, std::vector<int64_t>& sc_ptr,
                          std::vector<int>& sc_pos);

}  // namespace gdsw
