/*
 * libfind -- FIND selected inversion on AMD MI355X (gfx950).
 *
 * For every energy E of a batch, with the n x n matrix
 *     A(E) = E*I - H - Sigma_L(E) - Sigma_R(E)         (n = Nx*Ny)
 * the library returns diag(G), diag(G<), and the nearest-neighbour entries of
 * G and G< with the bond currents, where G = A^{-1} and
 * G< = G Sigma< G^dagger (paper, Sec. 1, NEGF equations; Sec. 3.1 for diag G<,
 * Sec. 3.2 for the off-diagonal entries used for current density).  The
 * method is FIND: a nested-dissection upward pass over the basic cluster tree
 * (procedure updateBoundaryNodes), a downward pass over the complement
 * clusters (procedure updateAdjacentNodes), both by the Schur-complement
 * update of eq. (major-update) and the Sigma update of eq. (gless-update-rule),
 * followed by a per-leaf extraction (eq. (cd1)-(cd3) and eq. (gless-nn)),
 * as in procedure computeG<.
 *
 * Data conventions (all arrays dense, C order, complex = two doubles re,im):
 *   mesh node (x, y), x in [0,Nx) transverse, y in [0,Ny) transport,
 *   linear index i = y*Nx + x; contacts on the columns y = 0 (left, contact 0)
 *   and y = Ny-1 (right, contact 1).
 *   H          double [nst][Ny][Nx], nst = 3 (5-point) or 5 (9-point):
 *              [0] on-site H_ii, [1] H between (x,y),(x+1,y), [2] (x,y),(x,y+1),
 *              [3] (x,y),(x+1,y+1), [4] (x+1,y),(x,y+1).  H must be real
 *              symmetric (the stored value is used for both H_ij and H_ji).
 *   energies   complex [nE]   (E + i*eta, eta > 0)
 *   sigma      complex [nE][2][Nx][Nx]: sigma[e][c][a][b] = Sigma_c(row a, col b)
 *              (row-major inside each contact block; for the complex
 *              symmetric leads of a real transverse basis this equals the
 *              column-major layout)
 *   sigma_less complex [nE][2][Nx][Nx], same layout (Sigma<_c)
 *   diag_G, diag_Gless   complex [nE][Ny][Nx]
 *   bond_G, bond_Gless   complex [nE][nbonds]  (G_ij and G<_ij, i first node)
 *   bond_J               double  [nE][nbonds]  (J_{i->j} = 2 Re(H_ij G<_ji))
 *   Bonds are numbered family by family: x-bonds [Ny][Nx-1] (i=(x,y), j=(x+1,y)),
 *   y-bonds [Ny-1][Nx] (i=(x,y), j=(x,y+1)), and for 9-point meshes
 *   d+ bonds [Ny-1][Nx-1] (i=(x,y), j=(x+1,y+1)) and d- bonds [Ny-1][Nx-1]
 *   (i=(x+1,y), j=(x,y+1)).  find_n_bonds() gives nbonds.
 *
 * Memory and threading: every pointer passed to find_solve is a DEVICE
 * pointer on the current HIP device, owned by the caller; the library never
 * frees or keeps caller pointers past the call.  find_solve only enqueues work
 * on the given HIP stream (NULL = default stream) and returns; outputs are
 * valid once that stream has been synchronised.  A plan owns its device
 * workspace and tree maps (allocated on first use on a device); calls that
 * share a plan must be serialised by the caller (one stream at a time).
 * Graph capture: find_solve enqueues kernels and event waits only, so it may
 * be captured into a HIP graph, provided an eager find_solve of at least as
 * many energies ran first on the same device (nothing is allocated under
 * capture; otherwise FIND_E_ARG).  Buffers a captured solve references stay
 * valid until find_plan_destroy: a later eager solve that needs larger
 * buffers allocates new ones and keeps the old.
 * No function throws across this boundary; errors are returned as
 * find_status and described by find_last_error() (thread-local string).
 */
#ifndef FIND_H_
#define FIND_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct find_plan_s* find_plan;

typedef enum {
  FIND_OK = 0,
  FIND_E_ARG = 1,         /* invalid argument (sizes, NULL pointers, stencil) */
  FIND_E_NOMEM = 2,       /* device allocation failed / over budget            */
  FIND_E_SINGULAR = 3,    /* zero or tiny pivot met (see find_sync_status)      */
  FIND_E_DEVICE = 4,      /* HIP runtime error                                  */
  FIND_E_UNSUPPORTED = 5  /* shape beyond what the kernels support             */
} find_status;

typedef enum { FIND_PREC_FP64 = 0, FIND_PREC_MIXED = 1, FIND_PREC_MIXED_GLESS = 2 } find_precision;
typedef enum { FIND_CPLX_4M = 0, FIND_CPLX_3M = 1 } find_complex_mode;

/* Plan options; pass NULL for defaults.
 *   leaf          largest leaf-cluster side (default 8): the mesh is bisected
 *                 along its longer side (y on ties) until both sides <= leaf
 *                 (paper Sec. 2.1, the nested-dissection partition).
 *   precision     FIND_PREC_FP64 (default), FIND_PREC_MIXED or
 *                 FIND_PREC_MIXED_GLESS.  In FIND_PREC_MIXED the
 *                 Schur-complement and Sigma products of eq. (major-update)
 *                 and eq. (gless-update-rule) run in FP32 on MFMA (FP32
 *                 accumulation); in FIND_PREC_MIXED_GLESS only the Sigma
 *                 products of eq. (gless-update-rule) do (the G< part: W and
 *                 R), while U = A(B,B) - L A(S,B) stays FP64, so diag G is the
 *                 FP64 result and diag G< carries the FP32 rounding of the
 *                 Sigma products only.  In both, the LU of A(S,S), the L solve,
 *                 the final leaf blocks, every elimination of a cluster at
 *                 tree depth <= fp64_top_levels, and every elimination with
 *                 s >= 512 stay FP64.  Stored U/R blocks are FP64.
 *   max_energies  energies processed per internal pass (0 = chosen from the
 *                 workspace budget).
 *   fp64_top_levels  see precision (0 = default 2, negative = none).
 *   workspace_budget  device bytes the plan may hold (0 = three quarters of
 *                 the current device's memory, or 64 GiB where no device is
 *                 visible, e.g. for find_plan_footprint on a host without
 *                 one).  A solve of more energies than fit runs in passes of
 *                 equal size.
 *   complex_mode  real split of the complex Schur-complement and Sigma
 *                 products: FIND_CPLX_4M (default; four real products per
 *                 complex product) or FIND_CPLX_3M (three: ar br, ai bi and
 *                 (ar + ai)(br + bi)).  3M rounds differently, within the
 *                 same tolerances; flop counts stay at 8 per complex
 *                 multiply-add either way.
 *   symmetric     1 or 2 asserts that A is complex symmetric (H real
 *                 symmetric, Sigma_L and Sigma_R complex symmetric, as for
 *                 leads with a real transverse basis).  Every Schur
 *                 complement U is then complex symmetric (Prop. 1 of the
 *                 paper): with 1, only its lower triangle is formed and it is
 *                 stored packed by columns (column c holds rows c..b-1), and
 *                 readers take an upper entry from its mirror (s b^2 / 2
 *                 fewer complex multiply-adds per elimination; the flop model
 *                 of find_plan_flops follows).  R (anti-Hermitian when Sigma<
 *                 is) is then formed and stored whole.  With 2, R is halved
 *                 the same way (an upper entry read as minus the conjugate of
 *                 its mirror), so that the energy pool is about half that of
 *                 the general form (storage reduction of the symmetric U, and
 *                 of the anti-Hermitian R); the two computed triangles of R
 *                 round differently, and the mirrored R amplifies the rounding
 *                 of G< = G R G^dagger at energies near resonances (diag G<
 *                 relative errors up to ~1e-7 against ~1e-12, G unaffected).
 *                 The mirrored U itself costs a factor of a few in accuracy at
 *                 ill-conditioned energies (errors up to ~5e-10 where the
 *                 general form has 1e-10), so the general form is the
 *                 accurate default.  Inputs that break the assertion give
 *                 wrong results.  0 (default) = general, U and R whole.
 *   streams       energy groups solved concurrently inside one pass (0 or 1
 *                 = one, on the caller's stream; 2..4 = that many groups, each
 *                 on a stream of the plan, forked from and joined back to the
 *                 caller's stream with events, each with its own workspace),
 *                 so that one group's small late stages overlap another's.
 *                 Results do not depend on it.
 *   scattering    1: the solves add diagonal scattering self-energies on
 *                 every node (the paper's problem statement, Sec. 1, takes the
 *                 scattering self-energy as typically diagonal): Sigma_d is
 *                 subtracted from the diagonal of A and Sigma<_d added to the
 *                 diagonal of Sigma<, both passed to find_solve_scattering.  Every
 *                 node then carries Sigma<, so no front skips its W and R.
 *                 0 (default): contacts only, find_solve.
 *   half_leaves   1: the current density scheme of Sec. 4.3 (Fig. cd-opt):
 *                 only a checkerboard of leaves runs the leaf extraction and
 *                 final block, each keeping the ring of nodes around it and
 *                 returning the diagonal and bond entries of that ring too, so
 *                 that the other leaves need no extraction.  A leaf is added
 *                 to the checkerboard wherever a node or bond would otherwise
 *                 lie in no chosen leaf's kept set (always with 9-point
 *                 meshes, whose diagonal bonds inside a skipped leaf no
 *                 neighbour reaches; with leaves larger than 2 x 2 the
 *                 interior of a skipped leaf forces it in).  Results are
 *                 those of the default (every leaf); only the work differs.
 *                 0 (default): every leaf.
 *   no_contacts   1: a closed device, A = E I - H (- diag Sigma_d with
 *                 scattering): no contact self-energies, so the boundary
 *                 sets follow the stencil alone (the physical boundary of the
 *                 paper's Table NullBoundaryCost) and sigma / sigma_less may
 *                 be NULL (they are not read).  0 (default): contacts on the
 *                 columns y = 0 and y = Ny - 1. */
typedef struct {
  int leaf;
  int precision;
  int max_energies;
  int fp64_top_levels;
  size_t workspace_budget;
  int complex_mode;
  int symmetric;
  int streams;
  int scattering;
  int half_leaves;
  int no_contacts;
  int reserved[2];
} find_plan_opts;

/* Build the cluster tree, boundary sets, gather maps and level schedule for
 * an Nx x Ny mesh with a 5- or 9-point stencil and dense contact columns
 * (paper Sec. 2.1-2.2 for the trees and sets; procedure computeG<).  Host
 * only; device state is created on first find_solve.
 * Errors: FIND_E_ARG if Nx < 1, Ny < 1, stencil not 5/9, out == NULL,
 * or leaf < 1; FIND_E_UNSUPPORTED for more than 2^24 nodes, a front
 * (eliminated plus kept nodes of one elimination) of more than 4096 nodes,
 * or a final leaf block of more than 1024.  Fronts of 2049..4096 nodes
 * (contact columns of more than 1024 nodes join the separators: a 1024 x 256
 * 9-point mesh has fronts of 2808) run in launch configuration 7 only. */
find_status find_plan_create(int Nx, int Ny, int stencil, const find_plan_opts* opts,
                             find_plan* out);

/* Release the plan and all device memory it holds.  NULL is accepted. */
find_status find_plan_destroy(find_plan plan);

/* Device bytes one find_solve over nE energies holds (plan maps + energy
 * pool + elimination workspace), sized as find_solve sizes them on the
 * current device (its CU count; 256 CUs if no device is present); for
 * serving admission.  The pool holds, per energy, the U and R blocks of
 * every cluster (the storage of eq. (major-update) and eq.
 * (gless-update-rule)); buffers only grow, so a plan that ran a larger solve
 * holds more.  want_bonds selects the leaf extraction that also yields the
 * bond entries. */
find_status find_plan_footprint(find_plan plan, int nE, int want_bonds, size_t* bytes);

/* Algorithmic real flops per energy (8 per complex multiply-add): for each
 * elimination with s eliminated and b kept nodes, s^3/3 + 2 s^2 b + 3 s b^2
 * complex multiply-adds (the paper's operation counts, eq.
 * (basic-computation-cost) for U: LU of A(S,S), L = A(B,S) A(S,S)^-1, the
 * Schur update of eq. (major-update); eq. (gless-computation-cost) for R: the
 * two products of eq. (gless-update-rule) arranged as W = [-L, I] Sigma,
 * R = W [-L, I]^dagger), reduced by the exact zeros and the halved
 * triangles of the plan's form; plus 2 b'^3 for each
 * final leaf block of size b' (the inverse G and T = R G^dagger; the requested
 * entries of G< = G T are O(b') dot products each). */
find_status find_plan_flops(find_plan plan, int want_bonds, double* flops_per_energy);

/* Number of bonds (output length per energy of bond_G/bond_Gless/bond_J). */
int find_n_bonds(int Nx, int Ny, int stencil);

/* Enqueue the whole FIND solve for nE energies on `hip_stream`.
 * Inputs and outputs are device pointers in the layouts above.  diag_G and
 * diag_Gless are required; bond_G, bond_Gless and bond_J may each be NULL
 * (if all three are NULL the cheaper diagonal-only leaf extraction runs).
 * Errors: FIND_E_ARG (nE < 1, NULL required pointer), FIND_E_NOMEM,
 * FIND_E_DEVICE, FIND_E_UNSUPPORTED (a front larger than the kernels
 * handle).  Pivot breakdown is reported by find_sync_status. */
find_status find_solve(find_plan plan, int nE, const double* energies, const double* H,
                       const double* sigma, const double* sigma_less, double* diag_G,
                       double* diag_Gless, double* bond_G, double* bond_Gless, double* bond_J,
                       void* hip_stream);

/* find_solve for a plan created with opts.scattering = 1 (the diagonal
 * scattering self-energies of the introduction, e.g. electron-phonon):
 * A = E I - H - Sigma_L - Sigma_R - diag(Sigma_d) and Sigma< = Sigma<_L +
 * Sigma<_R + diag(Sigma<_d), with sigma_d and sigma_less_d complex
 * [nE][Ny][Nx] device arrays (node (x, y) at [e][y][x], like diag_G):
 * Sigma_d retarded (Im <= 0), Sigma<_d anti-Hermitian, i.e. purely
 * imaginary, for the symmetric form.  Both are read once per solve, before
 * the first elimination, on `hip_stream`.  Other arguments and errors as
 * find_solve; FIND_E_ARG also if the plan is not a scattering plan or
 * sigma_d or sigma_less_d is NULL (find_solve rejects scattering plans). */
find_status find_solve_scattering(find_plan plan, int nE, const double* energies, const double* H,
                                  const double* sigma, const double* sigma_less, const double* sigma_d,
                                  const double* sigma_less_d, double* diag_G, double* diag_Gless,
                                  double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream);

/* find_solve_scattering with, in addition, stencil-pattern (nearest-
 * neighbour) scattering self-energies, the general form of a local
 * self-energy (paper §1: the scattering self-energy is often, not always,
 * diagonal): A = E I - H - Sigma_L - Sigma_R - diag(Sigma_d) - Sigma_b and
 * Sigma< = ... + diag(Sigma<_d) + Sigma<_b.  sigma_b and sigma_less_b are
 * complex device arrays [nE][nst-1][Ny][Nx][2] laid out like H's bond planes
 * (plane k = 1 .. nst-1 of H is plane k-1 here) with two values per bond:
 * [..][y][x][0] is the entry (i, j) from the bond's first node i to its second
 * node j, [..][y][x][1] the entry (j, i) (the bond of H plane k at (x, y), as
 * described for H; entries of bonds that leave the mesh are not read).  For
 * the symmetric forms Sigma_b must be symmetric (equal entries for both
 * directions) and Sigma<_b anti-Hermitian.  bond_J stays 2 Re(H_ij G<_ji)
 * (the coherent part of the current).  Requires a scattering plan; every
 * pointer but the optional bond outputs must be non-NULL (zero arrays for an
 * absent diagonal part).  Other arguments and errors as
 * find_solve_scattering. */
find_status find_solve_scattering_bonds(find_plan plan, int nE, const double* energies, const double* H,
                                        const double* sigma, const double* sigma_less, const double* sigma_d,
                                        const double* sigma_less_d, const double* sigma_b,
                                        const double* sigma_less_b, double* diag_G, double* diag_Gless,
                                        double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): find_solve for
 * a contacts-only plan with every scratch buffer of the solve (energy pool,
 * elimination workspace, pivot status) taken from a fixed device array of
 * 512 MiB that the library holds on each device it runs on until the process
 * ends.  It calls no hipMalloc, hipFree or other allocating routine.
 * Preconditions: the plan's tables are on the current device, i.e. find_solve
 * (or find_plan_autotune) ran with this plan on this device before, else
 * FIND_E_ARG.  Energies are solved in passes of as many as fit the array
 * next to the nE status entries; if one energy of the plan does not fit
 * (e.g. more than about 1.2 energies' worth of a 128 x 128 mesh's U and R
 * blocks), FIND_E_NOMEM with the bytes needed.  It runs on `hip_stream` only
 * (opts.streams and profiling do not apply) with the plan's stage tiles, so
 * its results equal find_solve's.  Every call on a device shares that
 * device's array: calls that overlap in time on one device (on different
 * streams or host threads) race and give wrong results; find_sync_status
 * for such a call reads the array, so it must come before the next call on
 * the device.  Other arguments and errors as find_solve. */
find_status find_solve_noalloc(find_plan plan, int nE, const double* energies, const double* H,
                               const double* sigma, const double* sigma_less, double* diag_G, double* diag_Gless,
                               double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream);

/* Wait for `hip_stream`, then report FIND_E_SINGULAR if the last solve on
 * this plan met a zero or tiny pivot in the LU of some A(S,S) (eq.
 * (express-L)) or of a final leaf block (eq. (cd1)): |re| + |im| of the pivot
 * below 1e3 * eps * the largest |re| + |im| of that block (eps = 2^-52).  A
 * zero pivot is replaced by 1 so that the solve stays finite; a tiny one is
 * used as it is; the results of that energy are unreliable either way.  The
 * first such energy index is in find_last_error().  Else FIND_OK. */
find_status find_sync_status(find_plan plan, void* hip_stream);

/* Thread-local description of the last error of this thread. */
const char* find_last_error(void);

/* Instrumentation for roofline measurement.  While enabled, find_solve
 * records a HIP event pair on its stream around every elimination-stage
 * kernel launch, or, with several energy groups (streams > 1), around each
 * pass (inside a captured hipGraph the pairs are part of the graph and are
 * re-recorded by every replay).  find_plan_profile waits for the event pairs
 * of the most recent find_solve (or of the latest replay of a captured one)
 * and returns their summed elapsed milliseconds, their algorithmic flops (the
 * find_plan_flops model for the eliminations and energies each timed region
 * processed) and the number of elimination-stage kernel launches the solve
 * enqueued.  Any pointer argument may be NULL. */
find_status find_plan_set_profiling(find_plan plan, int enable);
find_status find_plan_profile(find_plan plan, double* kernel_ms, double* kernel_flops, int* launches);

/* Launch-shape autotuner (not a step of the method: it only picks how the
 * work of a stage is spread over workgroups and waves).  Each stage of the
 * plan (the eliminations of one tree level and pass, launched together) has a
 * launch configuration: 0..3 = one 256-thread workgroup per front with wave
 * tiles of 32x32, 32x16, 16x32 or 16x16 for the Schur products of eq.
 * (major-update) and eq. (gless-update-rule) (stages whose fronts exceed 512
 * nodes, and the final leaf blocks, have 0 only); 4 = one 64-thread workgroup
 * (a single wave) per front, for stages whose fronts have at most 128 nodes;
 * 5 = one 128-thread workgroup (two waves) per front, fronts of at most 256;
 * 6 = one 256-thread workgroup per front with 64x64 workgroup tiles whose
 * operands the four waves share through LDS, for the Schur products and the
 * LU trailing updates (stages whose fronts have at most 512 nodes, not the
 * final leaf blocks); 7 = one 512-thread workgroup (eight waves) per front and
 * one workgroup per compute unit, for stages with few large fronts (fronts of
 * up to 2048 nodes, not the final leaf blocks); 8 = final leaf blocks only
 * (diagonal outputs, blocks of at most 64 nodes with R_K supported on at most
 * 28): G = U_K^{-1} by Gauss-Jordan elimination with partial pivoting with the
 * whole block in registers, diag G< as quadratic forms over R_K's support.
 * Configurations 0..3 and 6 only decide which threads compute which part of
 * the same operations in the same order, so their results are bitwise the
 * same; 4, 5 and 7 factor fronts with other register panels (same
 * operations, other rounding); 8 inverts by another elimination order (other
 * rounding).
 *   find_plan_autotune runs one solve of the first min(nE, pass size)
 *   energies stage by stage, times every configuration of every stage `reps`
 *   times (reps < 1 means 2) with HIP events on `hip_stream`, keeps the
 *   fastest, and leaves that solve's diag G / diag G< in the outputs.  It
 *   synchronises the stream; FIND_E_ARG if the stream is being captured.
 *   A scattering plan is tuned on a solve with zero scattering self-energies
 *   (the same work: such a plan forms W and R on every front whatever their
 *   values), whose results the outputs then hold.
 *   find_plan_get_tiles copies min(cap, n_stages) configurations (stage
 *   order of find_plan_export) to tiles and the bit mask of the
 *   configurations each stage has to masks (either may be NULL), and stores
 *   the stage count in *n_stages.
 *   find_plan_set_tiles sets them (n must equal the stage count; each value
 *   must be a configuration the stage has, else FIND_E_ARG). */
find_status find_plan_autotune(find_plan plan, int nE, const double* energies, const double* H,
                               const double* sigma, const double* sigma_less, double* diag_G,
                               double* diag_Gless, int reps, void* hip_stream);
find_status find_plan_get_tiles(find_plan plan, int* tiles, int* masks, int cap, int* n_stages);
find_status find_plan_set_tiles(find_plan plan, const int* tiles, int n);

/* ---- Introspection (host only; for tests and tools) ---------------------- */
typedef struct {
  int Nx, Ny, stencil, leaf;
  int n_clusters, depth, n_leaves;
  int n_elims, n_stages, map_len;
  int n_leafout, n_outbonds, n_outnodes;
  int max_n, max_s, max_b;
  int64_t pool_per_energy; /* complex elements per energy */
  int reserved[8];
} find_plan_summary_t;

/* Field layout of one exported elimination record (int32 each). */
enum {
  FIND_EF_KIND = 0,    /* 0 = Schur elimination, 1 = final leaf block           */
  FIND_EF_S, FIND_EF_B, FIND_EF_N,
  FIND_EF_SRC0, FIND_EF_LD0, FIND_EF_SRC1, FIND_EF_LD1, /* pool offsets (complex), -1 = none */
  FIND_EF_DST,         /* pool offset of U (b x b); R follows at DST + b*b, or  */
                       /* at DST + b(b+1)/2 with U packed (symmetric forms)    */
  FIND_EF_MAP,         /* first entry of this elimination's map (n entries)    */
  FIND_EF_CLUSTER, FIND_EF_PHASE, FIND_EF_LEVEL,
  FIND_EF_RZERO,       /* 1: Sigma< vanishes on the front, so R = 0 (not formed) */
  FIND_EF_SSIG,        /* eliminated nodes carrying Sigma< (the first SSIG of S) */
  FIND_EF_BSIG,        /* 1: some kept node coupled to S carries Sigma<          */
  FIND_EF_BACT,        /* kept nodes coupled to S (the first BACT of B)          */
  FIND_EF_FIELDS
};
/* Phases: 0 upward, 1 downward, 2 leaf extraction, 3 final leaf block.
 * Map entries are (node, src, pos): global node id (-1 for none), source
 * 0/1 (pos = row in that source's b x b matrix) or 2 (original A / Sigma). */
/* Stage record: (first elim, count, phase, variant); variant 0 = diagonal
 * only, 1 = with bonds, -1 = both. */
/* Leaf-output record: (final elim, n_nodes, node_first, bond_first, n_bonds, variant).
 * Out-node entries: (global node, local index).  Out-bond entries:
 * (bond id, local i, local j, stencil array k, flat H index y*Nx+x). */
enum { FIND_SF_FIELDS = 4, FIND_LF_FIELDS = 6, FIND_ON_FIELDS = 2, FIND_OB_FIELDS = 5 };

find_status find_plan_summary(find_plan plan, find_plan_summary_t* out);
find_status find_plan_export(find_plan plan, int32_t* elims, int32_t* maps, int32_t* stages,
                             int32_t* leafout, int32_t* outnodes, int32_t* outbonds);

#ifdef __cplusplus
}
#endif
#endif /* FIND_H_ */
