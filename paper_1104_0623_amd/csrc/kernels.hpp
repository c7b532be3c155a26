// Device-side records and kernel launchers for the FIND elimination path.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace findmi {

// One elimination as the kernels see it (mirrors findmi::Elim).
struct ElimDev {
  int kind, s, b, n;
  long long src0, src1;   // pool offsets (complex) of source U matrices; R follows each U
  int ld0, ld1;
  long long dst;          // pool offset of the output U (b x b, or its packed lower triangle); R follows
  int map;                // first map entry
  int aux;                // final leaf block: index of its output record
  int f32;                // bit 0: U product in FP32, bit 1: W and R (Sigma) products in FP32
  int rzero;              // 1: Sigma< vanishes on the front: R = 0, only U is formed
  int ssig;               // eliminated nodes carrying Sigma< (the first ssig of S)
  int bsig;               // 1: some kept node coupled to S carries Sigma<
  int bact;               // kept nodes coupled to S (the first bact of B)
};

struct LeafOutDev { int elim_dst_lo, elim_dst_hi, bprime, n_nodes, node_first, bond_first, n_bonds, pad; };

struct StageArgs {
  const ElimDev* elims;   // this stage's records, sorted by decreasing cost
  int n_elims;
  int nE;                 // energies in this pass
  const int* map_node;    // global node id per map entry
  const int* map_srcpos;  // (src << 24) | pos per map entry
  const double2* energies;  // energies of this pass
  const double* H;        // [nst][Ny][Nx]
  const double2* sigma;   // sigma of this pass  [nE][2][Nx][Nx]
  const double2* sless;
  const double2* sscat;   // diagonal scattering Sigma of this pass [nE][Ny][Nx], or NULL
  const double2* slscat;  // and Sigma< (read by the node-diagonal pre-pass only)
  const double2* sbond;   // stencil-pattern scattering Sigma of this pass [nE][nst-1][Ny][Nx][2], or NULL
  const double2* slbond;  // and Sigma<
  long long onsite_off;   // pool offset (per energy) of the node diagonal E - H_ii - Sigma_d,i, then Sigma<_d,i
  double2* pool;          // pool of this pass, energy stride pool_stride
  long long pool_stride;
  double2* ws;            // per-slot workspace
  long long ws_stride;
  int Nx, Ny, nst;
  int* status;            // per energy of this pass: 1 = zero or tiny pivot met
  int sym;                // bit 0: U complex symmetric, bit 1: R anti-Hermitian; each such block is
                          // formed and stored as its packed lower triangle
  int contacts;           // 1: contact self-energies on the columns y = 0 and y = Ny - 1 (sigma, sless read)
};

struct OutArgs {
  const LeafOutDev* leaves;
  const int* outnode;     // (node, local) pairs
  const int* outbond;     // (bond, li, lj, k, hflat) records
  const double* H;
  int n_bonds;
  double2* diag_G;        // outputs of this pass (already offset to the first energy)
  double2* diag_Gless;
  double2* bond_G;
  double2* bond_Gless;
  double* bond_J;
};

// rows per thread of the register-resident LU panel needed for a front of size n
inline int panel_rpt(int n) { return n <= 256 ? 1 : n <= 512 ? 2 : n <= 1024 ? 4 : 8; }
constexpr int kMaxFront = 4096;        // eight-wave form, eight panel rows a thread
constexpr int kFourWaveMaxFront = 2048; // every other form of a Schur elimination, and final blocks
constexpr int kThreads = 256;

// Stage launchers (one per kernel family; see kernels.hip).  tc: wave tile of
// the Schur products (0..3; families with 4 or 8 panel rows per thread take
// tc = 0 only), kTileWave: one 64-thread workgroup (a single wave) per front,
// for stages whose fronts have at most kWaveMaxFront nodes, kTileTwoWave:
// one 128-thread workgroup per front (fronts of at most kTwoWaveMaxFront
// nodes), or kTileWg: 64x64 workgroup tiles whose operands the four waves
// share through LDS (Schur products and LU trailing updates; fronts of at
// most 512 nodes), or kTileEight: one 512-thread workgroup per front and per
// CU, for stages with few, large fronts.  kTileGJ (final leaf blocks only):
// Gauss-Jordan inversion of the whole block in registers, for blocks of at most
// 64 nodes with R_K supported on at most 28 of them and diagonal outputs.
// cm: 0 = 4M, 1 = 3M complex products.
constexpr int kTileConfigs = 9;
constexpr int kTileWave = 4;       // one wave (64 threads) per front
constexpr int kTileTwoWave = 5;    // two waves (128 threads) per front
constexpr int kTileWg = 6;         // 64x64 workgroup tiles staged through LDS
constexpr int kTileEight = 7;      // eight waves (512 threads) per front, one workgroup per CU
constexpr int kTileGJ = 8;         // final blocks: register-resident Gauss-Jordan (see k_final_gj)
constexpr int kGjMaxB = 64, kGjMaxRs = 28;
constexpr int kEightWaveThreads = 512;
constexpr int kWaveMaxFront = 128;
constexpr int kTwoWaveMaxFront = 256;
// workgroups resident where one 256-thread workgroup is, for a configuration
inline int groups_per_slot(int tc) { return tc == kTileWave ? 4 : tc == kTileTwoWave ? 2 : 1; }
// workgroups a stage launches with configuration tc on a device with `slots`
// 256-thread slots (three per CU); the workgroup-tile form is compiled for
// two workgroups per CU
inline long long stage_grid_groups(long long slots, int tc) {
  if (tc == kTileEight) return slots / 3;   // one eight-wave workgroup per CU
  if (tc == kTileGJ) return slots;          // three 256-thread workgroups per CU
  return tc == kTileWg ? slots * 2 / 3 : slots * groups_per_slot(tc);
}
#define FIND_CAT_(a, b) a##b
#define FIND_CAT(a, b) FIND_CAT_(a, b)
hipError_t launch_stage_r1(const StageArgs& a, int tc, int cm, int grid, hipStream_t st);
hipError_t launch_stage_r2(const StageArgs& a, int tc, int cm, int grid, hipStream_t st);
hipError_t launch_stage_r48(const StageArgs& a, int rpt, int tc, int cm, int grid, hipStream_t st);
hipError_t launch_stage_w(const StageArgs& a, int rpt, int cm, int grid, hipStream_t st);
hipError_t launch_stage_w2(const StageArgs& a, int rpt, int cm, int grid, hipStream_t st);
hipError_t launch_stage_w8(const StageArgs& a, int rpt, int cm, int grid, hipStream_t st);
hipError_t launch_final(const StageArgs& a, const OutArgs& o, int rpt, int grid, hipStream_t st);
hipError_t launch_final_w(const StageArgs& a, const OutArgs& o, int rpt, int grid, hipStream_t st);
hipError_t launch_final_w2(const StageArgs& a, const OutArgs& o, int rpt, int grid, hipStream_t st);
hipError_t launch_final_gj(const StageArgs& a, const OutArgs& o, int grid, hipStream_t st);
// panel rows per thread of the one- and two-wave forms
inline int wave_rpt(int n) { return n <= 64 ? 1 : 2; }
inline int wave2_rpt(int n) { return n <= 128 ? 1 : 2; }
inline int wave8_rpt(int n) { return n <= 512 ? 1 : n <= 1024 ? 2 : n <= 2048 ? 4 : 8; }
// bit mask of the tile configurations a stage with fronts of at most maxn nodes has;
// gj_ok: a final stage whose blocks fit k_final_gj (at most kGjMaxB nodes, R_K
// on at most kGjMaxRs, no bond outputs)
// (fronts of more than kFourWaveMaxFront nodes: the eight-wave form only, and
// no final stage; 0 = no configuration)
inline int stage_tile_mask(int maxn, bool final_stage, bool gj_ok = false) {
  if (maxn > kFourWaveMaxFront) return final_stage ? 0 : 1 << kTileEight;
  int m = final_stage ? 1 : (panel_rpt(maxn) <= 2 ? (0xf | 1 << kTileWg) : 1);
  if (final_stage && gj_ok) m |= 1 << kTileGJ;
  if (!final_stage) m |= 1 << kTileEight;
  if (maxn <= kWaveMaxFront) m |= 1 << kTileWave;
  if (maxn <= kTwoWaveMaxFront) m |= 1 << kTileTwoWave;
  return m;
}
inline hipError_t launch_stage(const StageArgs& a, int maxn, int tc, int cm, int grid, hipStream_t st) {
  if (tc == kTileEight) return launch_stage_w8(a, wave8_rpt(maxn), cm, grid, st);
  if (maxn > kFourWaveMaxFront) return hipErrorInvalidValue;
  if (tc == kTileWave) return maxn <= kWaveMaxFront ? launch_stage_w(a, wave_rpt(maxn), cm, grid, st) : hipErrorInvalidValue;
  if (tc == kTileTwoWave)
    return maxn <= kTwoWaveMaxFront ? launch_stage_w2(a, wave2_rpt(maxn), cm, grid, st) : hipErrorInvalidValue;
  switch (panel_rpt(maxn)) {
    case 1: return launch_stage_r1(a, tc, cm, grid, st);
    case 2: return launch_stage_r2(a, tc, cm, grid, st);
    default: return launch_stage_r48(a, panel_rpt(maxn), tc, cm, grid, st);
  }
}
inline hipError_t launch_final_tc(const StageArgs& a, const OutArgs& o, int maxn, int tc, int grid, hipStream_t st) {
  if (maxn > kFourWaveMaxFront) return hipErrorInvalidValue;
  if (tc == kTileGJ) return launch_final_gj(a, o, grid, st);
  if (tc == kTileWave) return maxn <= kWaveMaxFront ? launch_final_w(a, o, wave_rpt(maxn), grid, st) : hipErrorInvalidValue;
  if (tc == kTileTwoWave)
    return maxn <= kTwoWaveMaxFront ? launch_final_w2(a, o, wave2_rpt(maxn), grid, st) : hipErrorInvalidValue;
  return tc == 0 ? launch_final(a, o, panel_rpt(maxn), grid, st) : hipErrorInvalidValue;
}

}  // namespace findmi
