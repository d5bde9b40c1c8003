// Runs the library's host set-up (reference element, connectivity, levels, face-node maps, point
// location) on a mesh read from raw files, so that a test can build it with AddressSanitizer and
// UndefinedBehaviorSanitizer and compare the integer results with the oracle's.
//   usage: host_setup_driver DIR N N_LEVELS
//   reads  DIR/verts.f64 (n_vert x 3), DIR/etov.i64 (K x 4), DIR/rho.f64, DIR/c.f64 (K), DIR/pts.f64 (n x 3)
//   writes DIR/EToE.i32, DIR/EToF.i8, DIR/level.i8, DIR/vmapP.i32, DIR/elem.i64
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_1506_00907_amd/csrc/setup.hpp"

template <class T>
static std::vector<T> load(const std::string &path) {
  std::vector<T> v;
  FILE *f = std::fopen(path.c_str(), "rb");
  if (!f) {
    std::fprintf(stderr, "cannot open %s\n", path.c_str());
    std::exit(2);
  }
  std::fseek(f, 0, SEEK_END);
  const long n = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  v.resize((size_t)n / sizeof(T));
  if (!v.empty() && std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) std::exit(2);
  std::fclose(f);
  return v;
}

template <class T>
static void save(const std::string &path, const std::vector<T> &v) {
  FILE *f = std::fopen(path.c_str(), "wb");
  if (!f || (!v.empty() && std::fwrite(v.data(), sizeof(T), v.size(), f) != v.size())) std::exit(2);
  std::fclose(f);
}

int main(int argc, char **argv) {
  if (argc != 4) return 2;
  const std::string dir = argv[1];
  const int N = std::atoi(argv[2]), nl = std::atoi(argv[3]);
  const auto verts = load<double>(dir + "/verts.f64");
  const auto etov = load<int64_t>(dir + "/etov.i64");
  const auto rho = load<double>(dir + "/rho.f64");
  const auto c = load<double>(dir + "/c.f64");
  const auto pts = load<double>(dir + "/pts.f64");
  const int64_t K = (int64_t)etov.size() / 4, nv = (int64_t)verts.size() / 3, np = (int64_t)pts.size() / 3;
  dgrtm::RefOps ref;
  dgrtm::build_ref(N, ref);
  dgrtm::HostMesh m;
  std::string err = dgrtm::mesh_build(m, N, nv, verts.data(), K, etov.data(), nullptr, 2, ref);
  if (!err.empty()) {
    std::fprintf(stderr, "mesh_build: %s\n", err.c_str());
    return 3;
  }
  err = dgrtm::mesh_set_model(m, rho.data(), c.data(), nl, 0.15);
  if (!err.empty()) {
    std::fprintf(stderr, "mesh_set_model: %s\n", err.c_str());
    return 3;
  }
  std::vector<int32_t> vmapP((size_t)K * 4 * ref.Nfp);
  dgrtm::mesh_vmapP(m, ref, vmapP.data());
  std::vector<int64_t> elem((size_t)np);
  std::vector<double> rst((size_t)np * 3);
  if (np) dgrtm::locate_points(m, np, pts.data(), elem.data(), rst.data());
  save(dir + "/EToE.i32", m.EToE);
  save(dir + "/EToF.i8", m.EToF);
  save(dir + "/level.i8", m.level);
  save(dir + "/vmapP.i32", vmapP);
  save(dir + "/elem.i64", elem);
  return 0;
}
