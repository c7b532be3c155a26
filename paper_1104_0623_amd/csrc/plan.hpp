// Host-side FIND plan: cluster tree, boundary sets, elimination records with
// their gather maps, the level schedule, and the per-energy pool layout.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace findmi {

struct Rect { int x0, y0, w, h; };

struct Cluster {
  Rect r;
  int parent = -1, child[2] = {-1, -1}, sibling = -1;
  int depth = 0, height = 0;
  std::vector<int> B;    // boundary set B_C: nodes of C with a pattern-neighbour outside C
  std::vector<int> Bc;   // B_{C-bar}: nodes outside C with a pattern-neighbour in C
  // per node of B (Bc): 1 if its row of the stored R_C (R_{C-bar}) may be non-zero
  std::vector<char> up_sig, dn_sig;
  int64_t up_off = -1;   // pool offset of (U_C, R_C)
  int64_t dn_off = -1;   // pool offset of (U_{C-bar}, R_{C-bar})
  bool leaf() const { return child[0] < 0; }
};

enum Phase { PH_UP = 0, PH_DOWN = 1, PH_LEAF = 2, PH_FINAL = 3 };
enum Kind { K_SCHUR = 0, K_FINAL = 1 };
enum Src { SRC0 = 0, SRC1 = 1, SRC_ORIG = 2 };

struct Elim {
  int kind = K_SCHUR;
  int s = 0, b = 0, n = 0;
  int64_t src_off[2] = {-1, -1};
  int src_ld[2] = {0, 0};
  int64_t dst = -1;
  int map = 0;
  int cluster = -1, phase = 0, level = 0;
  // 1: Sigma< vanishes on every node of the front (an upward-pass cluster that
  // touches neither contact column), so R = 0 and only U is formed
  int rzero = 0;
  // number of eliminated nodes whose rows of the assembled Sigma_g may be
  // non-zero; they come first in S, and the rows of Sigma_g of the other
  // s - ssig eliminated nodes (and their columns) are exactly zero
  int ssig = 0;
  // 1: some kept node carries Sigma< (its row of Sigma_g may be non-zero)
  int bsig = 0;
  // kept nodes coupled to S (the first bact of B): the rows and columns of
  // A_g and Sigma_g between the other kept nodes and S are exactly zero, so
  // the elimination leaves their rows and columns of U and R unchanged
  int bact = 0;
};

struct Stage { int first, count, phase, variant; };
struct LeafOut { int elim, n_nodes, node_first, bond_first, n_bonds, variant; };
struct OutBond { int bond, li, lj, k, hflat; };

struct Plan {
  int Nx = 0, Ny = 0, stencil = 5, leaf = 8;
  // diagonal scattering self-energies on every node: every node carries Sigma<
  bool scattering = false;
  // leaf extraction on a checkerboard of leaves whose kept sets cover the ring
  // around them (current density from half of the leaves)
  bool half_leaves = false;
  // contact self-energies on the columns y = 0 and y = Ny - 1 (false: a closed
  // device, A = E I - H, no contact coupling in the sets)
  bool contacts = true;
  // stored triangles: bit 0 = each U (complex symmetric) kept as its lower
  // triangle packed by columns, bit 1 = each R (anti-Hermitian) likewise;
  // R follows U in its slot either way
  int pack = 0;
  // pool offset (per energy) of the node diagonal: A_ii of the original matrix
  // without its contact part (E - H_ii - Sigma_d,i), then Sigma<_d,i ([2][Ny][Nx])
  int64_t onsite_off = 0;
  std::vector<Cluster> cl;
  int depth = 0, n_leaves = 0;
  std::vector<Elim> elims;
  std::vector<int> map_node, map_src, map_pos;
  std::vector<Stage> stages;
  std::vector<LeafOut> leafout;
  std::vector<int> outnode_node, outnode_local;
  std::vector<OutBond> outbonds;
  int64_t pool_per_energy = 0;
  int max_n = 0, max_s = 0, max_b = 0;
  int n_bonds = 0;
  // per energy: [halved triangles, as elim_flops' sym: 0 none, 1 U, 3 U and R][variant 0/1]
  double flops[4][2] = {};
};

int count_bonds(int Nx, int Ny, int stencil);
// Builds the plan; returns an empty string on success, else a message.
std::string build_plan(int Nx, int Ny, int stencil, int leaf, Plan& P, bool scattering = false,
                       bool half_leaves = false, bool contacts = true, int pack = 0);
// complex elements of a stored b x b block: whole, or a packed lower triangle
inline int64_t block_elems(int64_t b, bool packed) { return packed ? b * (b + 1) / 2 : b * b; }
// sym: bit 0 = only half of U formed, bit 1 = only half of R formed
double elim_flops(const Elim& e, int sym = 0);

}  // namespace findmi
