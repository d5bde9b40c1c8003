// Host-side set-up of the DG operators, mesh connectivity and multi-rate levels (FP64).
//
// Reference element: nodal Lagrange basis on warp-and-blend nodes
// (Np = (N+1)(N+2)(N+3)/6), differentiation matrices D_r, D_s, D_t and the
// lifting matrix (nodal-DG section and appendix).  Built from the orthonormal
// simplex basis (collapsed coordinates + Jacobi polynomials), so that
// M^{-1} = V V^T and LIFT = V V^T E.
//
// Reference tetrahedron V0=(-1,-1,-1), V1=(1,-1,-1), V2=(-1,1,-1), V3=(-1,-1,1);
// faces 0..3 are t=-1 (V0V1V2), s=-1 (V0V1V3), r+s+t=-1 (V1V2V3), r=-1 (V0V2V3).
// Node (i,j,l), i+j+l<=N, has integer barycentric weights (N-i-j-l,i,j,l) on
// (V0..V3), ordered l slowest, then j, then i fastest.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dgrtm {

constexpr int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
constexpr int kFaceOpp[4] = {3, 2, 0, 1};

inline int n_nodes(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
inline int n_face_nodes(int N) { return (N + 1) * (N + 2) / 2; }

struct RefOps {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<int> lat;          // Np x 4 barycentric integer weights
  std::vector<double> r, s, t;   // node coordinates
  std::vector<double> V;         // Np x Np Vandermonde (orthonormal basis), row = node
  std::vector<double> Dr, Ds, Dt;  // Np x Np, row-major
  std::vector<double> LIFT;      // Np x 4Nfp, row-major
  std::vector<int> Fmask;        // 4 x Nfp
  // face-node matching: for our face f, neighbour face f2 and vertex permutation code p
  // (our face vertex a maps to the neighbour's face vertex perm[p][a]),
  // nbr_index[((f*4+f2)*6+p)*Nfp + i] = index on the neighbour face of our face node i.
  std::vector<int> nbr_index;
};

// the six permutations of three face vertices
constexpr int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

void build_ref(int N, RefOps &ref);
// orthonormal simplex basis values at (r,s,t): out[Np]
void basis_at(const RefOps &ref, double r, double s, double t, double *out);
// small dense helpers (row-major)
bool invert(int n, std::vector<double> &A);

struct HostMesh {
  int N = 0;
  int64_t K = 0, n_vert = 0;
  std::vector<double> verts;       // n_vert x 3
  std::vector<int64_t> etov;       // K x 4 (oriented)
  std::vector<int32_t> EToE;       // K x 4 (self on boundary)
  std::vector<int8_t> EToF;        // K x 4
  std::vector<int8_t> face_perm;   // K x 4, permutation code 0..5 (0 on boundary)
  std::vector<int8_t> bc;          // K x 4 (0 interior, 1 rigid, 2 transparent, 3 free)
  std::vector<double> geo;         // K x 9: rx ry rz sx sy sz tx ty tz
  std::vector<double> J;           // K
  // model
  bool has_model = false;
  std::vector<double> rho, c;      // K
  std::vector<int8_t> level;       // K, 1 = coarsest
  int L = 1;
  double dt_local = 0.0;
  // level-sorted layout: sorted position -> user element (-1 for padding), user -> sorted
  std::vector<int64_t> sorted_to_user, user_to_sorted;
  std::vector<int64_t> lev_begin;  // begin of level l's padded segment (index l-1 for level l); finest first
  std::vector<int64_t> lev_count;  // real elements per level
  int64_t Ktot = 0;                // padded total
};

std::string mesh_build(HostMesh &m, int N, int64_t n_vert, const double *xyz, int64_t K,
                       const int64_t *etov, const int8_t *face_bc, int bc_default, const RefOps &ref);
std::string mesh_set_model(HostMesh &m, const double *rho, const double *c, int n_levels_max, double cfl);
// user-order global node ids of the neighbour face nodes (K x 4 x Nfp), vmapP in the paper's sense
void mesh_vmapP(const HostMesh &m, const RefOps &ref, int32_t *vmapP);
// point location: lowest element whose barycentric coordinates are all >= -1e-12; -1 if none
void locate_points(const HostMesh &m, int64_t n, const double *xyz, int64_t *elem, double *rst);

// record msg as this thread's last error (dgrtm_last_error) and return code
int32_t report_error(int32_t code, const std::string &msg);

}  // namespace dgrtm
