// Host-only driver of the map builder (paper_2606_01433_amd/csrc/maps.cpp) for
// sanitizer runs: reads a problem's integer arrays from a directory, builds the
// maps of every level exactly as the library's setup does (level mesh, maps,
// next level's mesh, recursion of section 2.2) and writes them back for
// comparison.  Built with -fsanitize=address,undefined by
// tests/test_host_maps_sanitized.py; nothing else uses it.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2606_01433_amd/csrc/maps.h"

template <typename T>
static std::vector<T> load(const std::string& path) {
  std::vector<T> v;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return v;
  std::fseek(f, 0, SEEK_END);
  const long bytes = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  v.resize(bytes / sizeof(T));
  if (!v.empty() && std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) v.clear();
  std::fclose(f);
  return v;
}

template <typename T, typename A>
static void store(const std::string& path, const std::vector<T, A>& v) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) return;
  if (!v.empty()) std::fwrite(v.data(), sizeof(T), v.size(), f);
  std::fclose(f);
}

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: maps_driver <in dir> <out dir>\n");
    return 2;
  }
  const std::string in = argv[1], out = argv[2];
  // meta: n, n_nodes, n_elem, levels, overlap, n_parts[levels - 1]
  const std::vector<int64_t> meta = load<int64_t>(in + "/meta.bin");
  if (meta.size() < 5) return 3;
  const int64_t n = meta[0];
  const int n_nodes = (int)meta[1], n_elem = (int)meta[2], levels = (int)meta[3], overlap = (int)meta[4];
  std::vector<int> n_parts(meta.begin() + 5, meta.end());
  const std::vector<int> node_dof = load<int>(in + "/node_dof.bin");
  const std::vector<int> elem_node = load<int>(in + "/elem_node.bin");
  const std::vector<int> elem_pdof = load<int>(in + "/elem_pdof.bin");
  const std::vector<int> elem_part = load<int>(in + "/elem_part.bin");
  std::vector<gdsw::LevelMesh> meshes(1);
  std::string err = gdsw::build_level1_mesh(n, n_nodes, node_dof.data(), n_elem, elem_node.data(),
                                            elem_pdof.data(), elem_part.data(), n_parts[0], meshes[0]);
  if (!err.empty()) {
    std::fprintf(stderr, "%s\n", err.c_str());
    return 4;
  }
  int written = 0;
  for (int l = 1; l < levels; ++l) {
    gdsw::LevelMaps m;
    gdsw::build_domains(meshes[l - 1], overlap, m);
    gdsw::build_maps(meshes[l - 1], overlap, m);
    const std::string p = out + "/L" + std::to_string(l) + "_";
    store(p + "dom_ptr.bin", m.dom_ptr);
    store(p + "dom.bin", m.dom);
    store(p + "int_ptr.bin", m.int_ptr);
    store(p + "inter.bin", m.inter);
    store(p + "ent_ptr.bin", m.ent_ptr);
    store(p + "ent_nodes.bin", m.ent_nodes);
    store(p + "col_entity.bin", m.col_entity);
    store(p + "owner.bin", m.owner);
    std::vector<int64_t> sc_ptr;
    std::vector<int> sc_pos;
    err = gdsw::scatter_lists(m, meshes[l - 1].n_dof, true, sc_ptr, sc_pos);
    if (!err.empty()) return 5;
    store(p + "sc_ptr.bin", sc_ptr);
    ++written;
    if (l == levels - 1 || n_parts[l] == 1) break;
    const std::vector<int> parent = load<int>(in + "/parent" + std::to_string(l) + ".bin");
    meshes.emplace_back();
    err = gdsw::build_next_mesh(meshes[l - 1], m, parent.data(), n_parts[l], meshes[l]);
    if (!err.empty()) {
      std::fprintf(stderr, "%s\n", err.c_str());
      return 6;
    }
  }
  std::printf("levels written: %d\n", written);
  return 0;
}
