// FIND elimination kernels for gfx950 (FP64 complex).
//
// One workgroup (256 threads, four wave64s) owns one (energy, elimination)
// work item at a time and walks a persistent loop over the stage's items.
// For an item with s eliminated and b kept nodes (n = s + b) it
//   1. assembles the tall block [A_g(S,S); A_g(B,S)] of the front in [S ; B]
//      order from the stored U/R blocks of its sources and the original
//      A / Sigma (the block assembly of procedures updateBoundaryNodes and
//      updateAdjacentNodes; Sec. 3.1 for the Sigma blocks); the remaining
//      blocks are gathered the same way when the products read them,
//   2. LU-factors the tall block [A(S,S); A(B,S)] with partial pivoting over
//      the S rows only (register-resident panels, MFMA trailing updates); the
//      B rows of the result hold L21 = A(B,S) U11^{-1},
//   3. forms L = A(B,S) A(S,S)^{-1} = L21 L11^{-1} P (eq. (express-L)),
//      written with its columns in the front's S order,
//   4. computes U = A(B,B) - L A(S,B) (eq. (major-update)), and
//   5. R of eq. (gless-update-rule), Sigma(B,B) - L Sigma(S,B)
//      - Sigma(B,S) L^dagger + L Sigma(S,S) L^dagger, as
//      R = W(:,B) - W(:,S) L^dagger with W = [-L, I] Sigma.  Sigma_g vanishes
//      outside the rows and columns of the nodes that carry Sigma<; the plan
//      puts the q eliminated ones (S_q) first in S, so W(:,S) = 0 outside S_q,
//      and the kernel forms W_q = W(:,S_q) = Sigma(B,S_q) - L_q Sigma(S_q,S_q)
//      and R = Sigma(B,B) - [L_q | W_q] [Sigma(S_q,B) ; L_q^dagger], with
//      L_q = L(:,S_q) (the Sigma(S_q,B) half is skipped when no kept node
//      carries Sigma<).
// Kept nodes that share no source, stencil bond or contact column with S
// (placed last in B by the plan; leaf extraction only) have zero rows and
// columns of A_g(B,S) and Sigma_g(B,S): steps 1-5 run over the first bact
// kept nodes, and U and R keep A_g(B,B), Sigma_g(B,B) for the others.
// The row permutation P is never applied to the front: the LU reads row
// perm[k] for the k-th pivot, and the L solve stores column k at perm[k].
// Complex products run on v_mfma_f64_16x16x4_f64 as four real products
// (re*re - im*im, re*im + im*re); in the mixed forms the U product (bit 0 of
// ElimDev::f32) and the Sigma products (bit 1) may run on
// v_mfma_f32_16x16x4_f32 instead.
#include "kernels.hpp"

#include <climits>
#include <type_traits>

namespace findmi {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// c - a*b as four fused multiply-adds
__device__ __forceinline__ double2 cfms(double2 c, double2 a, double2 b) {
  return make_double2(fma(a.y, b.y, fma(-a.x, b.x, c.x)), fma(-a.y, b.x, fma(-a.x, b.y, c.y)));
}
// 1 / a with one division
__device__ __forceinline__ double2 cinv(double2 a) {
  const double rd = 1.0 / (a.x * a.x + a.y * a.y);
  return make_double2(a.x * rd, -a.y * rd);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }

// Entries of the original A = E I - H - Sigma_L - Sigma_R and of Sigma<,
// addressed by node coordinates (x, y) (no integer division).
// BONDS: the plan's solve passes stencil-pattern scattering self-energies
// (compiled separately, so that the gathers of every other solve keep their
// registers)
template <bool BONDS>
struct OrigT {
  const double* H;
  const double2* sig;
  const double2* sless;
  const double2* D;     // [2][Ny][Nx] of this energy: E - H_ii - Sigma_d,i, then Sigma<_d,i
  int Nx, Ny, nst;
  int scat;             // 1: diagonal scattering self-energies present (Sigma<_d read from D)
  int contacts;         // 1: contact self-energies on the columns y = 0 and y = Ny - 1
  // stencil-pattern scattering self-energies of this energy, laid out like
  // H's bond planes with two values per bond ([nst-1][Ny][Nx][2]: from the
  // bond's first node to its second, then back); read only with BONDS
  const double2* sb;
  const double2* slb;

  // The bond between i = (xi, yi) and j = (xj, yj), i != j: its plane k of H
  // (1 .. nst-1; 0 if the nodes are not stencil neighbours), the index of its
  // entry in the plane, and whether i is the bond's first node.
  __device__ int bond(int xi, int yi, int xj, int yj, int& idx, bool& fwd) const {
    const int dx = xj - xi, dy = yj - yi;
    fwd = true;
    if (dy == 0) {
      if (dx == 1) { idx = yi * Nx + xi; return 1; }
      if (dx == -1) { idx = yj * Nx + xj; fwd = false; return 1; }
      return 0;
    }
    if (dx == 0) {
      if (dy == 1) { idx = yi * Nx + xi; return 2; }
      if (dy == -1) { idx = yj * Nx + xj; fwd = false; return 2; }
      return 0;
    }
    if (nst == 5) {
      if (dx == 1 && dy == 1) { idx = yi * Nx + xi; return 3; }
      if (dx == -1 && dy == -1) { idx = yj * Nx + xj; fwd = false; return 3; }
      if (dx == -1 && dy == 1) { idx = yi * Nx + xj; return 4; }                // i=(x+1,y) first, j=(x,y+1)
      if (dx == 1 && dy == -1) { idx = yj * Nx + xi; fwd = false; return 4; }   // i=(x,y+1), j=(x+1,y) first
    }
    return 0;
  }
  // entry (i, j) of a bond self-energy array (zero unless the nodes are
  // stencil neighbours)
  __device__ double2 bond_value(const double2* b, int xi, int yi, int xj, int yj) const {
    int idx;
    bool fwd;
    const int k = bond(xi, yi, xj, yj, idx, fwd);
    return k ? b[(((size_t)(k - 1) * Nx * Ny + idx) << 1) + (fwd ? 0 : 1)] : zero2();
  }
  // H_ij for i = (xi, yi), j = (xj, yj), i != j (the bond lookup above,
  // written out with the plane offsets folded in)
  __device__ double hval(int xi, int yi, int xj, int yj) const {
    const int dx = xj - xi, dy = yj - yi;
    const int plane = Nx * Ny;
    if (dy == 0) return dx == 1 ? H[plane + yi * Nx + xi] : dx == -1 ? H[plane + yj * Nx + xj] : 0.0;
    if (dx == 0) return dy == 1 ? H[2 * plane + yi * Nx + xi] : dy == -1 ? H[2 * plane + yj * Nx + xj] : 0.0;
    if (nst == 5) {
      if (dx == 1 && dy == 1) return H[3 * plane + yi * Nx + xi];
      if (dx == -1 && dy == -1) return H[3 * plane + yj * Nx + xj];
      if (dx == -1 && dy == 1) return H[4 * plane + yi * Nx + xj];  // i=(x+1,y), j=(x,y+1)
      if (dx == 1 && dy == -1) return H[4 * plane + yj * Nx + xi];  // i=(x,y+1), j=(x+1,y)
    }
    return 0.0;
  }
  // A_ij
  __device__ double2 a(int xi, int yi, int xj, int yj) const {
    double2 av = zero2();
    const int dx = xj - xi, dy = yj - yi;
    if (dx == 0 && dy == 0) av = D[yi * Nx + xi];
    else if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) {
      av.x = -hval(xi, yi, xj, yj);
      if constexpr (BONDS) {
        const double2 t = bond_value(sb, xi, yi, xj, yj);
        av.x -= t.x; av.y -= t.y;
      }
    }
    if (contacts && dy == 0) {
      if (yi == 0) { const double2 t = sig[xi * Nx + xj]; av.x -= t.x; av.y -= t.y; }
      if (yi == Ny - 1) { const double2 t = sig[Nx * Nx + xi * Nx + xj]; av.x -= t.x; av.y -= t.y; }
    }
    return av;
  }
  // Sigma<_ij (non-zero only between two nodes of one contact column, and,
  // with scattering self-energies, on the diagonal and between stencil
  // neighbours)
  __device__ double2 s(int xi, int yi, int xj, int yj) const {
    double2 sv = zero2();
    if (scat && xi == xj && yi == yj) sv = D[Nx * Ny + yi * Nx + xi];
    if constexpr (BONDS) {
      if (xi != xj || yi != yj) {
        const double2 u = bond_value(slb, xi, yi, xj, yj);
        sv.x += u.x; sv.y += u.y;
      }
    }
    if (contacts && yi == yj) {
      if (yi == 0) { const double2 u = sless[xi * Nx + xj]; sv.x += u.x; sv.y += u.y; }
      if (yi == Ny - 1) { const double2 u = sless[Nx * Nx + xi * Nx + xj]; sv.x += u.x; sv.y += u.y; }
    }
    return sv;
  }
};

// Operand chunks of the 64x64 workgroup-tile products (gemm_wg): two
// buffers of an A chunk (8 k x 64 rows) and a B chunk (64 columns x 8 k, rows
// padded to 9 so that the 16 lanes reading one k of 16 columns hit distinct
// banks).
struct WgLds { double2 a[2][8][64]; double2 b[2][64][9]; };
struct NoWgLds {};

// Shared memory of one workgroup of NT threads working on fronts of at most
// MAXN nodes.  Four-wave workgroups on fronts of at most 512 nodes also hold
// the workgroup-tile staging buffers (three such workgroups fit one CU).
template <int NT, int MAXN>
struct LdsT {
  static constexpr int kNT = NT, kW = NT / 64;
  int node[MAXN];          // (y << 16) | x of each front row
  int srcpos[MAXN];
  int perm[MAXN];
  // pivot exchange, double-buffered by column parity: each wave's best
  // candidate key and the contents of its row
  unsigned long long candv[2][kW];
  double2 candrow[2][kW][16];
  double2 tri[16 * 16];
  double2 tinv[16 * 16];
  unsigned long long red[kW];   // per-wave partial maxima (norm of the pivot block)
  typename std::conditional<(NT == 256 && MAXN <= 512), WgLds, NoWgLds>::type wg;
};
template <class LDS>
constexpr bool has_wg() { return std::is_same<decltype(LDS::wg), WgLds>::value; }

// Stored b x b blocks of the pool: whole (column-major, ld b), or, in the
// symmetric forms, the lower triangle packed by columns (column c holds rows
// c .. b - 1 and starts at c b - c (c - 1) / 2).  U (complex symmetric) reads
// an upper entry as its mirror, R (anti-Hermitian) as minus the conjugate of
// its mirror.  R follows U in its slot.
__device__ __forceinline__ size_t tri_off(int r, int c, int b) {
  return (size_t)c * b - (((size_t)c * (c - 1)) >> 1) + (r - c);
}
__device__ __forceinline__ size_t block_size(int b, bool packed) {
  return packed ? ((size_t)b * (b + 1)) >> 1 : (size_t)b * b;
}
// element of entry (r, c) of a stored block (one load whatever the layout)
__device__ __forceinline__ size_t blk_index(int b, int r, int c, bool packed) {
  return packed ? tri_off(max(r, c), min(r, c), b) : (size_t)c * b + r;
}
__device__ __forceinline__ double2 read_u(const double2* U, int b, int r, int c, bool packed) {
  return U[blk_index(b, r, c, packed)];
}
__device__ __forceinline__ double2 read_r(const double2* R, int b, int r, int c, bool packed) {
  const double2 v = R[blk_index(b, r, c, packed)];
  return packed && r < c ? make_double2(-v.x, v.y) : v;
}
// store of entry (r, c) of a formed block; with a packed block only r >= c is kept
__device__ __forceinline__ void write_blk(double2* X, int b, int r, int c, bool packed, double2 v) {
  if (!packed) X[(size_t)c * b + r] = v;
  else if (r >= c) X[tri_off(r, c, b)] = v;
}

// Entries of the assembled front A_g / Sigma_g of one elimination, by front
// row/column (local [S ; B] index): the block of a source cluster's stored U
// (or R) when both indices come from that source, else the original A (or
// Sigma<) between the two mesh nodes.
template <bool BONDS>
struct FrontT {
  const int* node;     // LDS: (y << 16) | x
  const int* srcpos;   // LDS: (source << 24) | position
  const double2* U0;
  const double2* U1;
  int ld0, ld1;
  OrigT<BONDS> o;
  int sym;             // bit 0: sources hold U as a packed lower triangle, bit 1: R likewise

  __device__ double2 a(int r, int c) const {
    const int spr = srcpos[r], spc = srcpos[c];
    const int sr = spr >> 24;
    if (sr == (spc >> 24) && sr < 2)
      return read_u(sr ? U1 : U0, sr ? ld1 : ld0, spr & 0xffffff, spc & 0xffffff, sym & 1);
    const int gr = node[r], gc = node[c];
    return o.a(gr & 0xffff, gr >> 16, gc & 0xffff, gc >> 16);
  }
  __device__ double2 s(int r, int c) const {
    const int spr = srcpos[r], spc = srcpos[c];
    const int sr = spr >> 24;
    if (sr == (spc >> 24) && sr < 2) {
      const int ld = sr ? ld1 : ld0;
      const double2* R = (sr ? U1 : U0) + block_size(ld, sym & 1);
      return read_r(R, ld, spr & 0xffffff, spc & 0xffffff, sym & 2);
    }
    const int gr = node[r], gc = node[c];
    return o.s(gr & 0xffff, gr >> 16, gc & 0xffff, gc >> 16);
  }
};

// Visit (r, c) for r < nr, c < nc with the block's threads, column-major
// order inside a column, without integer division.
template <int NT, class F>
__device__ __forceinline__ void for_each_rc(int nr, int nc, F&& f) {
  constexpr int LNT = NT == 64 ? 6 : NT == 128 ? 7 : NT == 256 ? 8 : 9;
  static_assert((1 << LNT) == NT, "workgroup of 64, 128, 256 or 512 threads");
  const int lg = nr <= 1 ? 0 : 32 - __clz(nr - 1);
  const int lgr = lg < LNT ? lg : LNT;
  const int rmask = (1 << lgr) - 1, cstep = NT >> lgr;
  const int rr = threadIdx.x & rmask, cc = threadIdx.x >> lgr;
  for (int c = cc; c < nc; c += cstep)
    for (int r = rr; r < nr; r += rmask + 1) f(r, c);
}

// Visit (r, c) for r < nr, c < nc, column-major element order dealt to the
// threads in turn, NB elements per thread per round: the NB values are all
// fetched (get(r, c), independent loads) before any is consumed
// (put(r, c, v)), so that gathers from global memory overlap instead of
// waiting one by one.
template <int NT, int NBAT, class G, class P>
__device__ __forceinline__ void gather_rc(int nr, int nc, G&& get, P&& put) {
  if (nr <= 0 || nc <= 0) return;
  const int total = nr * nc;
  const int dc = NT / nr, dr = NT - dc * nr;         // advance of one round step (NT elements)
  int c0 = int(threadIdx.x) / nr, r0 = int(threadIdx.x) - c0 * nr;
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * NBAT) {
    double2 v[NBAT];
    int rr[NBAT], cc[NBAT];
    int r = r0, c = c0;
#pragma unroll
    for (int u = 0; u < NBAT; ++u) {
      rr[u] = r; cc[u] = c;
      v[u] = (e0 + u * NT < total) ? get(r, c) : make_double2(0.0, 0.0);
      r += dr; c += dc;
      if (r >= nr) { r -= nr; ++c; }
    }
#pragma unroll
    for (int u = 0; u < NBAT; ++u)
      if (e0 + u * NT < total) put(rr[u], cc[u], v[u]);
    r0 = r; c0 = c;
  }
}

// C(M x N) <- Cinit - A(M x K) B(K x N), complex.  Each wave computes one
// (16 TM) x (16 TN) output tile at a time on MFMA (four real products per
// complex product); operands are fetched PD k-steps ahead of use.  With F32
// the operands are rounded to FP32 and the product accumulates in FP32 on
// v_mfma_f32_16x16x4_f32; Cinit and the result stay FP64.
template <bool F32> struct MfmaT;
template <> struct MfmaT<false> {
  typedef double e; typedef d4 acc;
  static __device__ __forceinline__ acc mac(e a, e b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // D layout of the f64 16x16x4 MFMA: lane l, register q -> row 4q + l/16, column l%16
  static __device__ __forceinline__ int drow(int q, int lk) { return 4 * q + lk; }
};
template <> struct MfmaT<true> {
  typedef float e; typedef f4 acc;
  static __device__ __forceinline__ acc mac(e a, e b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // D layout of the f32 16x16x4 MFMA: lane l, register q -> row 4(l/16) + q, column l%16
  static __device__ __forceinline__ int drow(int q, int lk) { return 4 * lk + q; }
};

template <int NT, bool F32, int TM, int TN, bool C3, class LA, class LB, class LC, class SC>
__device__ __forceinline__ void gemm_tiles(int M, int N, int K, int tri, LA loadA, LB loadB, LC loadC, SC storeC) {
  typedef MfmaT<F32> T;
  typedef typename T::e E;
  constexpr int PD = 1;
  constexpr int NACC = C3 ? 3 : 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tm = (M + 16 * TM - 1) / (16 * TM), tn = (N + 16 * TN - 1) / (16 * TN);
  const int lr = lane & 15, lk = lane >> 4;
  const int nk = (K + 3) >> 2;
  int mine = -1;   // tiles are dealt to the waves in turn, skipped ones excluded
  for (int t = 0; t < tm * tn; ++t) {
    const int r0 = (t % tm) * 16 * TM, c0 = (t / tm) * 16 * TN;
    // tri > 0: tiles wholly inside columns < tri and strictly above the
    // diagonal are not formed (the caller mirrors them)
    if (c0 + 16 * TN <= tri && c0 >= r0 + 16 * TM) continue;
    if (++mine % (NT / 64) != wave) continue;
    // 4M: acc[0] = Re, acc[1] = Im.  3M: acc[0] = sum aR bR, acc[1] = sum aI bI,
    // acc[2] = sum (aR + aI)(bR + bI); Re = acc0 - acc1, Im = acc2 - acc0 - acc1.
    typename T::acc acc[NACC][TM][TN];
#pragma unroll
    for (int h = 0; h < NACC; ++h)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[h][i][j][q] = 0;
    E aR[PD + 1][TM], aI[PD + 1][TM], bR[PD + 1][TN], bI[PD + 1][TN];
    auto fetch = [&](int slot, int ks) {
      const int kk = 4 * ks + lk;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = r0 + 16 * i + lr;
        const double2 v = (r < M && kk < K) ? loadA(r, kk) : zero2();
        aR[slot][i] = E(v.x); aI[slot][i] = E(v.y);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = c0 + 16 * j + lr;
        const double2 v = (c < N && kk < K) ? loadB(kk, c) : zero2();
        bR[slot][j] = E(v.x); bI[slot][j] = E(v.y);
      }
    };
#pragma unroll
    for (int p = 0; p < PD; ++p) fetch(p, p);
    for (int ks = 0; ks < nk; ks += PD + 1) {
#pragma unroll
      for (int u = 0; u <= PD; ++u) {
        if (ks + u < nk) {
          fetch((u + PD) % (PD + 1), ks + u + PD);
          if constexpr (C3) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
              for (int j = 0; j < TN; ++j) {
                acc[0][i][j] = T::mac(aR[u][i], bR[u][j], acc[0][i][j]);
                acc[1][i][j] = T::mac(aI[u][i], bI[u][j], acc[1][i][j]);
              }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
              for (int j = 0; j < TN; ++j)
                acc[2][i][j] = T::mac(aR[u][i] + aI[u][i], bR[u][j] + bI[u][j], acc[2][i][j]);
          } else {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
              for (int j = 0; j < TN; ++j) {
                acc[0][i][j] = T::mac(aR[u][i], bR[u][j], acc[0][i][j]);
                acc[1][i][j] = T::mac(aR[u][i], bI[u][j], acc[1][i][j]);
              }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
              for (int j = 0; j < TN; ++j) {
                acc[0][i][j] = T::mac(-aI[u][i], bI[u][j], acc[0][i][j]);
                acc[1][i][j] = T::mac(aI[u][i], bR[u][j], acc[1][i][j]);
              }
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = r0 + 16 * i + T::drow(q, lk), c = c0 + 16 * j + lr;
          if (r < M && c < N) {
            const double2 v = loadC(r, c);
            double re, im;
            if constexpr (C3) {
              const double p0 = double(acc[0][i][j][q]), p1 = double(acc[1][i][j][q]);
              re = p0 - p1;
              im = double(acc[2][i][j][q]) - p0 - p1;
            } else {
              re = double(acc[0][i][j][q]);
              im = double(acc[1][i][j][q]);
            }
            storeC(r, c, make_double2(v.x - re, v.y - im));
          }
        }
  }
}

template <int NT, class LA, class LB, class LC, class SC>
__device__ __forceinline__ void gemm_sub(int M, int N, int K, LA loadA, LB loadB, LC loadC, SC storeC) {
  if (N <= 16) gemm_tiles<NT, false, 2, 1, false>(M, N, K, 0, loadA, loadB, loadC, storeC);
  else gemm_tiles<NT, false, 2, 2, false>(M, N, K, 0, loadA, loadB, loadC, storeC);
}

// C(M x N) <- Cinit - A(M x K) B(K x N), complex FP64, with 64x64 workgroup
// tiles: the four waves of a 256-thread workgroup stage A (64 x 8) and B
// (8 x 64) chunks through LDS (double-buffered, one barrier per chunk) and
// each wave computes one 32x32 quarter of the tile on MFMA.  Every entry sees
// the same MFMA sequence as with 32x32 wave tiles, so the two give identical
// results; the operand traffic per output is half.  tri as in gemm_tiles, at
// the granularity of the workgroup tile.  All threads of the workgroup call it.
template <class LA, class LB, class LC, class SC>
__device__ __forceinline__ void gemm_wg(WgLds& S, int M, int N, int K, int tri, LA loadA, LB loadB, LC loadC,
                                        SC storeC) {
  typedef MfmaT<false> T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int tm = (M + 63) >> 6, tn = (N + 63) >> 6;
  const int nc = (K + 7) >> 3;
  // staged elements of this thread: A (row ar, k ak and ak + 4), B (k bk,
  // columns bc and bc + 32); consecutive threads walk A down a column and B
  // along k, the contiguous directions of the operands
  const int ar = tid & 63, ak = tid >> 6;
  const int bk = tid & 7, bc = tid >> 3;
  for (int t = 0; t < tm * tn; ++t) {
    const int r0 = (t % tm) * 64, c0 = (t / tm) * 64;
    if (c0 + 64 <= tri && c0 >= r0 + 64) continue;
    d4 acc[2][2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[h][i][j][q] = 0;
    double2 ra[2], rb[2];
    auto gload = [&](int kc) {
      const int k0 = kc * 8;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = r0 + ar, k = k0 + ak + 4 * u;
        ra[u] = (r < M && k < K) ? loadA(r, k) : zero2();
        const int c = c0 + bc + 32 * u, kb = k0 + bk;
        rb[u] = (c < N && kb < K) ? loadB(kb, c) : zero2();
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        S.a[buf][ak + 4 * u][ar] = ra[u];
        S.b[buf][bc + 32 * u][bk] = rb[u];
      }
    };
    __syncthreads();   // readers of the previous tile's last chunk are done
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kc = 0; kc < nc; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nc) gload(kc + 1);
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        double aR[2], aI[2], bR[2], bI[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const double2 v = S.a[buf][4 * ks + lk][32 * wr + 16 * i + lr];
          aR[i] = v.x; aI[i] = v.y;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double2 v = S.b[buf][32 * wc + 16 * j + lr][4 * ks + lk];
          bR[j] = v.x; bI[j] = v.y;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[0][i][j] = T::mac(aR[i], bR[j], acc[0][i][j]);
            acc[1][i][j] = T::mac(aR[i], bI[j], acc[1][i][j]);
          }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[0][i][j] = T::mac(-aI[i], bI[j], acc[0][i][j]);
            acc[1][i][j] = T::mac(aI[i], bR[j], acc[1][i][j]);
          }
      }
      if (kc + 1 < nc) lstore(buf ^ 1);
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = r0 + 32 * wr + 16 * i + T::drow(q, lk), c = c0 + 32 * wc + 16 * j + lr;
          if (r < M && c < N) {
            const double2 v = loadC(r, c);
            storeC(r, c, make_double2(v.x - acc[0][i][j][q], v.y - acc[1][i][j][q]));
          }
        }
  }
}

// The Schur-complement products of an elimination, with the wave tile picked
// per stage (TC: 0 = 32x32, 1 = 32x16, 2 = 16x32, 3 = 16x16; 16-wide where N
// <= 16) and the 4M or 3M real split of the complex product (C3).  The tile
// only decides which wave computes which output block: every entry sees the
// same k-order, so the result does not depend on TC.
template <int NT, bool F32, int TC, bool C3, class LDS, class LA, class LB, class LC, class SC>
__device__ __forceinline__ void gemm_schur(LDS& L, int M, int N, int K, int tri, LA loadA, LB loadB, LC loadC,
                                           SC storeC) {
  if constexpr (TC == kTileWg && !F32 && !C3 && has_wg<LDS>()) {
    gemm_wg(L.wg, M, N, K, tri, loadA, loadB, loadC, storeC);
  } else {
    // (the workgroup tile has an FP64 4M form only; others take 32x32 wave tiles)
    constexpr int TM = (TC == 0 || TC == 1 || TC == kTileWg) ? 2 : 1;
    constexpr int TN = (TC == 0 || TC == 2 || TC == kTileWg) ? 2 : 1;
    if (TN == 2 && N <= 16) gemm_tiles<NT, F32, TM, 1, C3>(M, N, K, tri, loadA, loadB, loadC, storeC);
    else gemm_tiles<NT, F32, TM, TN, C3>(M, N, K, tri, loadA, loadB, loadC, storeC);
  }
}

// Inverse of the w x w unit-lower triangle held below the diagonal of L.tri
// (row-major, tri[i*16+j] = L_ij for i > j), written to L.tinv (zero outside
// w x w).  Thread j < 16 forward-substitutes column j of L^{-1}.  The caller
// has synchronised after writing L.tri; this function ends with a barrier.
template <class LDS>
__device__ __forceinline__ void tri_inverse_unit_lower(LDS& L, int w) {
  const int j = threadIdx.x;
  if (j < 16) {
    double2 y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double2 v = (i == j && i < w) ? make_double2(1.0, 0.0) : zero2();
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < i) v = cfms(v, L.tri[i * 16 + k], y[k]);
      y[i] = (i < w) ? v : zero2();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) L.tinv[i * 16 + j] = y[i];
  }
  __syncthreads();
}

// Pivot search key: the bits of a non-negative magnitude with the low
// kKeyBits replaced by kKeyRows - 1 - row.  Non-negative doubles order as their bit
// patterns, so the largest key (as an unsigned integer) is the largest
// magnitude (to within 2^-40 relative), ties going to the lowest row; every
// key of a row < kMaxFront is > 0.
constexpr int kKeyBits = 13, kKeyRows = 1 << kKeyBits;
static_assert(2 * kMaxFront <= kKeyRows, "pivot key row field too narrow");
typedef unsigned long long u64;
__device__ __forceinline__ u64 pivot_key(double mag, int row) {
  return ((u64)__double_as_longlong(mag) & ~(u64)(kKeyRows - 1)) | (u64)(kKeyRows - 1 - row);
}

// DPP move of a 64-bit value between lanes of a row of 16 (quad_perm or mirror).
template <int CTRL>
__device__ __forceinline__ u64 dpp_u64(u64 x) {
  const int lo = __builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(x >> 32), (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return ((u64)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ u64 readlane_u64(u64 x, int l) {
  const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return ((u64)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ u64 umax64(u64 a, u64 b) { return a > b ? a : b; }
// Maximum over the wave, returned to every lane: within rows of 16 by DPP
// (swap neighbours, swap pairs, half-row mirror, row mirror), then across the
// four rows by lane reads.
__device__ __forceinline__ u64 wave_max(u64 x) {
  x = umax64(x, dpp_u64<0xB1>(x));    // quad_perm [1,0,3,2]
  x = umax64(x, dpp_u64<0x4E>(x));    // quad_perm [2,3,0,1]
  x = umax64(x, dpp_u64<0x141>(x));   // row_half_mirror
  x = umax64(x, dpp_u64<0x140>(x));   // row_mirror
  return umax64(umax64(readlane_u64(x, 0), readlane_u64(x, 16)), umax64(readlane_u64(x, 32), readlane_u64(x, 48)));
}

// Pivot threshold of a front: kPivotRel * eps * ||A(S,S)||, with the norm
// taken as the largest |re| + |im| over the block (the measure the pivot
// search compares).  Each thread passes the maximum over the entries it
// assembled; the workgroup maximum is formed here.  Called by every thread;
// it ends with the barrier that publishes the assembled block.
constexpr double kPivotRel = 1e3;
template <class LDS>
__device__ __forceinline__ double pivot_threshold(LDS& L, double part) {
  const u64 w = wave_max((u64)__double_as_longlong(part));   // non-negative doubles order as integers
  if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = w;
  __syncthreads();
  u64 m = L.red[0];
#pragma unroll
  for (int k = 1; k < LDS::kW; ++k) m = umax64(m, L.red[k]);
  return kPivotRel * 2.220446049250313e-16 * __longlong_as_double((long long)m);
}

// Sum over the wave, returned to every lane (same pattern as wave_max).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  return __longlong_as_double((long long)dpp_u64<CTRL>((u64)__double_as_longlong(x)));
}
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  x += dpp_f64<0x140>(x);
  const u64 b = (u64)__double_as_longlong(x);
  return (__longlong_as_double((long long)readlane_u64(b, 0)) + __longlong_as_double((long long)readlane_u64(b, 16))) +
         (__longlong_as_double((long long)readlane_u64(b, 32)) + __longlong_as_double((long long)readlane_u64(b, 48)));
}

// v of the lane at byte address src (4 x lane) of this wave
__device__ __forceinline__ double bperm_d(int src, double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src, int(b & 0xffffffff));
  const int hi = __builtin_amdgcn_ds_bpermute(src, int(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 bperm_d2(int src, double2 v) {
  return make_double2(bperm_d(src, v.x), bperm_d(src, v.y));
}

// Physical row of logical row r of a front whose first s rows are pivoted.
__device__ __forceinline__ int prow(const int* pm, int s, int r) { return r < s ? pm[r] : r; }

// Blocked LU with partial pivoting (pivots searched among rows < s only) of
// the tall n x s block of FA (column-major, ld n).  Rows are never moved:
// perm[k] is the physical row holding logical row k (k < s; rows >= s are
// never pivoted), so every access to a pivot-eligible row goes through perm,
// and at the end perm[k] is the original row that became the k-th pivot.  Outer blocks of NB2 columns; inside a
// block, panels of NB columns are brought up to date left-looking from the
// block's earlier panels, factored in registers (rows spread over the
// threads), and their U rows formed; the rest of the matrix gets one
// MFMA trailing update per outer block.  Returns true if a pivot was zero or
// below thr in magnitude (|re| + |im|); a zero pivot is replaced by 1 so that
// the factorization stays finite, a tiny one is kept.
template <int RPT, int NB, bool WG, class LDS>
__device__ __forceinline__ bool tall_lu(LDS& L, double2* FA, int n, int s, double thr) {
  constexpr int NT = LDS::kNT;
  constexpr int NB2 = LDS::kNT >= 256 ? 64 : 32;   // outer block (columns per trailing update)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int* pm = L.perm;
  bool singular = false;
  for (int K0 = 0; K0 < s; K0 += NB2) {
    const int KE = min(s, K0 + NB2);
    for (int k0 = K0; k0 < KE; k0 += NB) {
      const int kb = min(NB, KE - k0);
      const int m = n - k0;          // panel rows
      const int ms = s - k0;         // pivot-eligible panel rows
      // (a) left-looking update of the panel by this block's earlier panels
      if (k0 > K0) {
        gemm_sub<NT>(m, kb, k0 - K0,
                 [=](int r, int k) { return FA[(size_t)(K0 + k) * n + prow(pm, s, k0 + r)]; },
                 [=](int k, int c) { return FA[(size_t)(k0 + c) * n + pm[K0 + k]]; },
                 [=](int r, int c) { return FA[(size_t)(k0 + c) * n + prow(pm, s, k0 + r)]; },
                 [=](int r, int c, double2 v) { FA[(size_t)(k0 + c) * n + prow(pm, s, k0 + r)] = v; });
        __syncthreads();
      }
      // (b) panel factorization with the panel in registers.  Register rows
      // stay with their threads: lg[q] is the logical panel row that register
      // row q currently stands for (pivoting trades logical labels, not data).
      // Columns >= kb and rows >= m are zero and stay zero.
      double2 P[RPT][NB];
      int lg[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int rho = tid + NT * q;
        lg[q] = rho;
#pragma unroll
        for (int j = 0; j < NB; ++j)
          P[q][j] = (rho < m && j < kb) ? FA[(size_t)(k0 + j) * n + prow(pm, s, k0 + rho)] : zero2();
      }
  #pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < kb) {
          const int buf = j & 1;
          // local candidate among this thread's pivot-eligible rows (logical
          // row in [j, ms)), as a packed key (see pivot_key); 0 = none
          u64 best = 0;
          int bq = 0;
  #pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (lg[q] >= j && lg[q] < ms) {
              const u64 v = pivot_key(fabs(P[q][j].x) + fabs(P[q][j].y), lg[q]);
              if (v > best) { best = v; bq = q; }
            }
          }
          const u64 wv = wave_max(best);
          // the owner of the wave's winner publishes columns j.. of its row
          if (best != 0 && best == wv) {
  #pragma unroll
            for (int q = 0; q < RPT; ++q)
              if (q == bq)
  #pragma unroll
                for (int jj = j; jj < NB; ++jj) L.candrow[buf][wave][jj] = P[q][jj];
          }
          if (lane == 0) L.candv[buf][wave] = wv;
          __syncthreads();
          // every thread picks the same winner
          u64 gk = L.candv[buf][0];
          int pw = 0;                                   // winning wave
  #pragma unroll
          for (int w = 1; w < LDS::kW; ++w) {
            const u64 o = L.candv[buf][w];
            if (o > gk) { gk = o; pw = w; }
          }
          int piv = kKeyRows - 1 - int(gk & (kKeyRows - 1));
          bool pvv = (gk >> kKeyBits) != 0;            // non-zero pivot magnitude
          if (piv < j || piv >= ms) { piv = j; pvv = false; }   // (logical row j is always eligible)
          // magnitude of the pivot (the key's bits above the row field)
          if (__longlong_as_double((long long)(gk & ~(u64)(kKeyRows - 1))) < thr) singular = true;
          if (tid == 0 && piv != j) {  // relabel: logical rows k0+j and k0+piv trade physical rows
            const int t = pm[k0 + j]; pm[k0 + j] = pm[k0 + piv]; pm[k0 + piv] = t;
          }
          // the pivot's register row becomes logical row j, the former j takes piv
  #pragma unroll
          for (int q = 0; q < RPT; ++q) lg[q] = lg[q] == piv ? j : (lg[q] == j ? piv : lg[q]);
          const double2* prow = L.candrow[buf][pw];
          double2 pv = prow[j];
          if (!pvv) { singular = true; pv = make_double2(1.0, 0.0); }
          const double2 inv = cinv(pv);
  #pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (lg[q] > j) {
              const double2 l = cmul(P[q][j], inv);
              P[q][j] = l;
  #pragma unroll
              for (int jj = j + 1; jj < NB; ++jj) P[q][jj] = cfms(P[q][jj], l, prow[jj]);
            }
          }
        }
      }
      __syncthreads();
      // write the panel back; keep its unit-lower top block
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (lg[q] < m) {
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (j < kb) FA[(size_t)(k0 + j) * n + prow(pm, s, k0 + lg[q])] = P[q][j];
          if (lg[q] < kb) {
#pragma unroll
            for (int j = 0; j < NB; ++j) L.tri[lg[q] * 16 + j] = P[q][j];
          }
        }
      }
      __syncthreads();
      // (d) U rows of this panel for the columns right of it
      if (k0 + kb < s) {
        const int cb = k0 + kb;
        if (k0 > K0)
          gemm_sub<NT>(kb, s - cb, k0 - K0,
                   [=](int r, int k) { return FA[(size_t)(K0 + k) * n + pm[k0 + r]]; },
                   [=](int k, int c) { return FA[(size_t)(cb + c) * n + pm[K0 + k]]; },
                   [=](int r, int c) { return FA[(size_t)(cb + c) * n + pm[k0 + r]]; },
                   [=](int r, int c, double2 v) { FA[(size_t)(cb + c) * n + pm[k0 + r]] = v; });
        tri_inverse_unit_lower(L, kb);
        const LDS* LL = &L;
        gemm_sub<NT>(kb, s - cb, kb,
                 [=](int r, int k) { double2 v = LL->tinv[r * 16 + k]; return make_double2(-v.x, -v.y); },
                 [=](int k, int c) { return FA[(size_t)(cb + c) * n + pm[k0 + k]]; },
                 [=](int r, int c) { return zero2(); },
                 [=](int r, int c, double2 v) { FA[(size_t)(cb + c) * n + pm[k0 + r]] = v; });
        __syncthreads();
      }
    }
    // (e) trailing update of rows KE..n, columns KE..s with the block's L and U
    if (KE < s) {
      auto la = [=](int r, int k) { return FA[(size_t)(K0 + k) * n + prow(pm, s, KE + r)]; };
      auto lb = [=](int k, int c) { return FA[(size_t)(KE + c) * n + pm[K0 + k]]; };
      auto lc = [=](int r, int c) { return FA[(size_t)(KE + c) * n + prow(pm, s, KE + r)]; };
      auto sc = [=](int r, int c, double2 v) { FA[(size_t)(KE + c) * n + prow(pm, s, KE + r)] = v; };
      if constexpr (WG && has_wg<LDS>()) gemm_wg(L.wg, n - KE, s - KE, KE - K0, 0, la, lb, lc, sc);
      else gemm_sub<NT>(n - KE, s - KE, KE - K0, la, lb, lc, sc);
      __syncthreads();
    }
  }
  return singular;
}

// X L11 = L21 for X = L21 L11^{-1} (L11 unit lower, L21 in FA rows s..n,
// columns 0..s, both in pivot order), stored as Lo(:, perm[k]) = X(:, k)
// (Lo is b x s with leading dimension b): Lo = X P = A(B,S) A(S,S)^{-1} with
// its columns in the front's S order.  FA rows s..n are overwritten.
template <class LDS>
__device__ __forceinline__ void trsm_right_unit_lower(LDS& L, double2* FA, double2* Lo, int n, int s, int b) {
  constexpr int NT = LDS::kNT;
  const int tid = threadIdx.x;
  const int nblk = (s + 15) / 16;
  const int* pm = L.perm;
  for (int J = nblk - 1; J >= 0; --J) {
    const int j0 = 16 * J, j1 = min(s, j0 + 16), w = j1 - j0;
    if (j1 < s) {
      gemm_sub<NT>(b, w, s - j1,
               [=](int r, int k) { return Lo[(size_t)pm[j1 + k] * b + r]; },
               [=](int k, int c) { return FA[(size_t)(j0 + c) * n + pm[j1 + k]]; },
               [=](int r, int c) { return FA[(size_t)(j0 + c) * n + s + r]; },
               [=](int r, int c, double2 v) { FA[(size_t)(j0 + c) * n + s + r] = v; });
    }
    {
      for (int t = tid; t < 256; t += NT) {
        const int i = t >> 4, jj = t & 15;
        L.tri[t] = (i < w && jj < w) ? FA[(size_t)(j0 + jj) * n + pm[j0 + i]] : zero2();
      }
    }
    __syncthreads();
    tri_inverse_unit_lower(L, w);
    {
      const LDS* LL = &L;
      gemm_sub<NT>(b, w, w,
               [=](int r, int k) { return FA[(size_t)(j0 + k) * n + s + r]; },
               [=](int k, int c) { double2 v = LL->tinv[k * 16 + c]; return make_double2(-v.x, -v.y); },
               [=](int r, int c) { return zero2(); },
               [=](int r, int c, double2 v) { Lo[(size_t)pm[j0 + c] * b + r] = v; });
    }
    __syncthreads();
  }
}

template <int RPT, int TC, int CM, int NT, int MAXN, bool BONDS = false>
__global__ __launch_bounds__(NT, (TC == kTileWg || NT == 512) ? 2 : 3) void k_stage(StageArgs a) {
  // panel columns held in registers (the eight-wave form, at two waves per
  // SIMD, has the registers for twice the panel width with four rows a thread)
  constexpr int NB = (NT == kEightWaveThreads && RPT >= 4) ? 32 / RPT : 16 / RPT;
  __shared__ LdsT<NT, MAXN> L;
  const int tid = threadIdx.x;
  const long long total = (long long)a.n_elims * a.nE;
  double2* FA = a.ws + (size_t)blockIdx.x * a.ws_stride;
  for (long long item = blockIdx.x; item < total; item += gridDim.x) {
    const int ei = int(item / a.nE), e = int(item % a.nE);
    const ElimDev E = a.elims[ei];
    const int s = E.s, b = E.b, n = E.n;
    // only the first ba kept nodes are coupled to S: the tall block, L, W_q and
    // the Schur corrections of U and R cover them (na = s + ba rows)
    const int ba = E.bact, na = s + ba;
    double2* Lo = FA + (size_t)na * s;  // FA: tall block na x s; Lo: L (ba x s, front column order)
    double2* W = Lo + (size_t)ba * s;   // W_q = W(:, S_q) (ba x q)
    double2* pool = a.pool + (size_t)e * a.pool_stride;
    for (int k = tid; k < n; k += NT) {
      const int g = a.map_node[E.map + k];
      const int y = g / a.Nx;
      L.node[k] = (y << 16) | (g - y * a.Nx);
      L.srcpos[k] = a.map_srcpos[E.map + k];
    }
    for (int k = tid; k < s; k += NT) L.perm[k] = k;
    __syncthreads();
    const FrontT<BONDS> fr{L.node, L.srcpos, pool + E.src0, pool + E.src1, E.ld0, E.ld1,
                   OrigT<BONDS>{a.H, a.contacts ? a.sigma + (size_t)e * 2 * a.Nx * a.Nx : nullptr,
                        a.contacts ? a.sless + (size_t)e * 2 * a.Nx * a.Nx : nullptr,
                        pool + a.onsite_off, a.Nx, a.Ny, a.nst, a.sscat != nullptr, a.contacts,
                        a.sbond ? a.sbond + (size_t)e * (a.nst - 1) * a.Nx * a.Ny * 2 : nullptr,
                        a.slbond ? a.slbond + (size_t)e * (a.nst - 1) * a.Nx * a.Ny * 2 : nullptr}, a.sym};
    // 1. assemble the tall block [A_g(S,S); A_g(B,S)]; the other blocks of A_g
    //    and all of Sigma_g are gathered from their sources by the products
    double amax = 0.0;   // this thread's largest |re| + |im| in A_g(S,S)
    gather_rc<NT, 8>(na, s, [&](int r, int c) { return fr.a(r, c); }, [&](int r, int c, double2 v) {
      FA[(size_t)c * na + r] = v;
      if (r < s) amax = fmax(amax, fabs(v.x) + fabs(v.y));
    });
    const double thr = pivot_threshold(L, amax);
    // 2. tall LU, 3. L = L21 L11^{-1}
    if (s > 0) {
      if (tall_lu<RPT, NB, TC == kTileWg>(L, FA, na, s, thr) && tid == 0) a.status[e] = 1;
      trsm_right_unit_lower(L, FA, Lo, na, s, ba);
    }
    // 4. U = A(B,B) - L A(S,B); 5. W_q and R (FP32 products in the mixed form,
    // FP64 otherwise)
    // U and R of this front, whole or as packed lower triangles
    const bool pu = a.sym & 1, pr = a.sym & 2;
    double2* Uo = pool + E.dst;
    double2* Ro = Uo + block_size(b, pu);
    const int q = E.ssig, q0 = E.bsig ? E.ssig : 0;
    auto lo_ = [=](int r, int k) { return Lo[(size_t)k * ba + r]; };
    auto bu = [=](int k, int c) { return fr.a(k, s + c); };
    auto cu = [=](int r, int c) { return fr.a(s + r, s + c); };
    auto su = [=](int r, int c, double2 v) { write_blk(Uo, b, r, c, pu, v); };
    auto bw = [=](int k, int c) { return fr.s(k, c); };
    auto cw = [=](int r, int c) { return fr.s(s + r, c); };
    auto sw = [=](int r, int c, double2 v) { W[(size_t)c * ba + r] = v; };
    // R = Sigma(B,B) - [L_q | W_q] [Sigma(S_q,B) ; L_q^dagger] (first half only when q0 = q)
    auto ar = [=](int r, int k) { return k < q0 ? Lo[(size_t)k * ba + r] : W[(size_t)(k - q0) * ba + r]; };
    auto br = [=](int k, int c) { return k < q0 ? fr.s(k, s + c) : conjd(Lo[(size_t)(k - q0) * ba + c]); };
    auto cr = [=](int r, int c) { return fr.s(s + r, s + c); };
    auto sr = [=](int r, int c, double2 v) { write_blk(Ro, b, r, c, pr, v); };
    // in the symmetric forms U (complex symmetric), and with sym bit 1 also R
    // (anti-Hermitian), is formed and stored as its lower triangle: tiles above
    // the diagonal are not formed, and readers take an upper entry from its
    // mirror below the diagonal
    const int tri = pu ? ba : 0, trir = pr ? ba : 0;
    auto products = [&](auto fu, auto fs) {
      constexpr bool FU = decltype(fu)::value, FS = decltype(fs)::value;
      gemm_schur<NT, FU, TC, CM == 1>(L, ba, ba, s, tri, lo_, bu, cu, su);
      if (E.rzero) {
        // Sigma< vanishes on this front: R = 0
        for_each_rc<NT>(b, b, [&](int r, int c) { write_blk(Ro, b, r, c, pr, zero2()); });
      } else {
        if (q > 0) gemm_schur<NT, FS, TC, CM == 1>(L, ba, q, q, 0, lo_, bw, cw, sw);
        __syncthreads();
        gemm_schur<NT, FS, TC, CM == 1>(L, ba, ba, q0 + q, trir, ar, br, cr, sr);
      }
    };
    // rows and columns of the kept nodes not coupled to S: U and R keep the
    // assembled A_g(B,B) and Sigma_g(B,B) there
    if (ba < b) {
      auto outside = [=](int r, int c, bool packed) { return (r >= ba || c >= ba) && (!packed || r >= c); };
      gather_rc<NT, 8>(b, b, [&](int r, int c) { return outside(r, c, pu) ? fr.a(s + r, s + c) : zero2(); },
                       [&](int r, int c, double2 v) { if (outside(r, c, pu)) write_blk(Uo, b, r, c, pu, v); });
      if (!E.rzero)
        gather_rc<NT, 8>(b, b, [&](int r, int c) { return outside(r, c, pr) ? fr.s(s + r, s + c) : zero2(); },
                         [&](int r, int c, double2 v) { if (outside(r, c, pr)) write_blk(Ro, b, r, c, pr, v); });
    }
    if (E.f32 == 3) products(std::true_type{}, std::true_type{});
    else if (E.f32 == 2) products(std::false_type{}, std::true_type{});
    else products(std::false_type{}, std::false_type{});
    __syncthreads();
  }
}

// Final leaf block (eq. (cd1) and eq. (gless-nn) on the kept set K = C u N):
// from the Schur complement U_K and its Sigma block R_K, G(K,K) = U_K^{-1} and
// G<(K,K) = G R_K G^dagger.  G comes out of the same tall LU + L solve as an
// elimination of [[U_K, I], [I, 0]]: the L block of that elimination is
// U_K^{-1}.  T = R_K G^dagger is formed once on MFMA; each requested entry of
// G< (the diagonal, and both orders of every bond) is then a dot product
// G(i,:) T(:,j) computed by one wave.  Outputs are written directly.
template <int RPT, int NT, int MAXN>
__global__ __launch_bounds__(NT, 3) void k_final(StageArgs a, OutArgs o) {
  constexpr int NB = 16 / RPT;  // panel columns held in registers
  __shared__ LdsT<NT, MAXN> L;
  const int tid = threadIdx.x;
  const long long total = (long long)a.n_elims * a.nE;
  double2* FA = a.ws + (size_t)blockIdx.x * a.ws_stride;
  const size_t nn = (size_t)a.Nx * a.Ny;
  for (long long item = blockIdx.x; item < total; item += gridDim.x) {
    const int ei = int(item / a.nE), e = int(item % a.nE);
    const ElimDev E = a.elims[ei];
    const LeafOutDev Lo = o.leaves[E.aux];
    const int bp = E.b, n = 2 * bp;
    double2* T = FA + (size_t)n * bp;             // bp x bp
    double2* pool = a.pool + (size_t)e * a.pool_stride;
    const bool pu = a.sym & 1, pr = a.sym & 2;
    const double2* Uin = pool + E.src0;             // U_K (bp x bp, whole or packed)
    const double2* Rin = Uin + block_size(bp, pu);  // R_K
    double2* G = pool + E.dst;                    // G(K,K), bp x bp
    for (int k = tid; k < bp; k += NT) L.perm[k] = k;
    double amax = 0.0;   // this thread's largest |re| + |im| in U_K
    gather_rc<NT, 8>(n, bp, [&](int r, int c) {
      return r < bp ? read_u(Uin, bp, r, c, pu)
                    : make_double2(r - bp == c ? 1.0 : 0.0, 0.0);
    }, [&](int r, int c, double2 v) {
      FA[(size_t)c * n + r] = v;
      if (r < bp) amax = fmax(amax, fabs(v.x) + fabs(v.y));
    });
    const double thr = pivot_threshold(L, amax);
    if (tall_lu<RPT, NB, false>(L, FA, n, bp, thr) && tid == 0) a.status[e] = 1;
    // G(:, perm[k]) = L(:, k): the L solve of the identity rows stores U_K^{-1}
    trsm_right_unit_lower(L, FA, G, n, bp, bp);
    // T = R_K G^dagger   (gemm_sub returns 0 - R G^dagger); R_K vanishes outside
    // its first rs rows and columns, so T has rs rows and the sum runs over rs
    const int rs = E.ssig;
    gemm_sub<NT>(rs, bp, rs,
             [=](int r, int k) { return read_r(Rin, bp, r, k, pr); },
             [=](int k, int c) { return conjd(G[(size_t)k * bp + c]); },
             [=](int r, int c) { return zero2(); },
             [=](int r, int c, double2 v) { T[(size_t)c * bp + r] = make_double2(-v.x, -v.y); });
    __syncthreads();
    // requested entries of G< = G T, one wave per entry: lanes split k, DPP sum
    const int lane = tid & 63, wave = tid >> 6;
    auto gless = [&](int i, int j) {
      double re = 0.0, im = 0.0;
      for (int k = lane; k < rs; k += 64) {
        const double2 p = cmul(G[(size_t)k * bp + i], T[(size_t)j * bp + k]);
        re += p.x; im += p.y;
      }
      return make_double2(wave_sum(re), wave_sum(im));
    };
    for (int q = wave; q < Lo.n_nodes; q += NT / 64) {
      const int node = o.outnode[2 * (Lo.node_first + q)];
      const int l = o.outnode[2 * (Lo.node_first + q) + 1];
      const double2 gl = gless(l, l);
      if (lane == 0) {
        o.diag_G[e * nn + node] = G[(size_t)l * bp + l];
        o.diag_Gless[e * nn + node] = gl;
      }
    }
    for (int q = wave; q < Lo.n_bonds; q += NT / 64) {
      const int* ob = o.outbond + 5 * (Lo.bond_first + q);
      const int bond = ob[0], li = ob[1], lj = ob[2], kk = ob[3], hf = ob[4];
      const size_t oi = (size_t)e * o.n_bonds + bond;
      if (o.bond_Gless) {
        const double2 v = gless(li, lj);
        if (lane == 0) o.bond_Gless[oi] = v;
      }
      if (o.bond_J) {
        const double2 v = gless(lj, li);
        if (lane == 0) o.bond_J[oi] = 2.0 * o.H[(size_t)kk * nn + hf] * v.x;
      }
      if (o.bond_G && lane == 0) o.bond_G[oi] = G[(size_t)lj * bp + li];
    }
    __syncthreads();
  }
}

// Final leaf blocks of at most kGjMax nodes whose R_K is supported on at most
// kGjRs of them, diagonal outputs only (eq. (cd1) and eq. (gless-nn) on K = C):
// G = U_K^{-1} by Gauss-Jordan elimination with partial pivoting, the whole
// 64 x 64 block in registers (thread t owns rows 4 (t % 16) .. + 3 and columns
// 4 (t / 16) .. + 3).  Step k takes the largest |re| + |im| of column k among
// the rows not pivoted yet (one DPP reduction by the 16 owners of the
// column, which are one row of lanes of one wave), publishes the column and
// the pivot through LDS (buffers by step parity, one barrier per step); every
// thread takes the pivot row's entries of its own columns from the lane of its
// wave that holds them, and updates its entries; pivot rows are
// relabelled, not moved, so that the block ends as G with its rows and
// columns permuted: entry (r, k) is G(step of row r, pivot row of step k).
// G(:, 0:rs) is then staged in LDS and diag G< = diag(G R_K G^dagger) is a
// quadratic form over the rs support rows per output node, four threads each.
// Nothing is written to the pool; results go straight to the outputs.
constexpr int kGjMax = kGjMaxB, kGjRs = kGjMaxRs;
struct GjLds {
  double2 pcol[2][kGjMax];   // column k of the current step, by step parity
  unsigned long long key[2];
  double2 pinv[2];           // reciprocal of the pivot
  unsigned long long red[4];
  int prowi[kGjMax];         // pivot row of each step
  int kinv[kGjMax];          // step at which each row was pivot
  double2 gd[kGjMax];        // diag G by local node
  double2 grs[kGjRs][kGjMax];  // G(a, b) for b < rs, at [b][a]
  double2 rs_[kGjRs][kGjRs];   // R_K(u, v) at [u][v]
};

template <int NT, int SYM>
__global__ __launch_bounds__(NT, 3) void k_final_gj(StageArgs a, OutArgs o) {
  static_assert(NT == 256, "one 256-thread workgroup per block (4 x 4 entries per thread)");
  __shared__ GjLds S;
  const int tid = threadIdx.x, lane = tid & 63;
  const int rb = tid & 15, cb = tid >> 4;
  const long long total = (long long)a.n_elims * a.nE;
  const size_t nn = (size_t)a.Nx * a.Ny;
  for (long long item = blockIdx.x; item < total; item += gridDim.x) {
    const int ei = int(item / a.nE), e = int(item % a.nE);
    const ElimDev E = a.elims[ei];
    const LeafOutDev Lo = o.leaves[E.aux];
    const int bp = E.b, rs = E.ssig;
    constexpr bool pu = SYM & 1, pr = SYM & 2;   // a.sym, as a template argument
    const double2* Uin = a.pool + (size_t)e * a.pool_stride + E.src0;   // U_K (whole or packed)
    const double2* Rin = Uin + block_size(bp, pu);                         // R_K
    double2 M[4][4];
    double amax = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * rb + i, c = 4 * cb + j;
        double2 v = make_double2(r == c ? 1.0 : 0.0, 0.0);
        if (r < bp && c < bp) {
          v = read_u(Uin, bp, r, c, pu);
          amax = fmax(amax, fabs(v.x) + fabs(v.y));
        }
        M[i][j] = v;
      }
    for (int t = tid; t < rs * rs; t += 256) {
      const int u = t % rs, v = t / rs;
      S.rs_[u][v] = read_r(Rin, bp, u, v, pr);
    }
    {
      const u64 w = wave_max((u64)__double_as_longlong(amax));
      if (lane == 0) S.red[tid >> 6] = w;
    }
    __syncthreads();
    const double thr = kPivotRel * 2.220446049250313e-16 *
                       __longlong_as_double((long long)umax64(umax64(S.red[0], S.red[1]), umax64(S.red[2], S.red[3])));
    u64 used = 0;          // rows pivoted so far (bit r)
    bool singular = false;
    // steps k = 4 kb + kj, kj unrolled so that column k is a register index
    for (int kb = 0; 4 * kb < bp; ++kb) {
      const bool owner = cb == kb;          // this thread holds column block kb
#pragma unroll
      for (int kj = 0; kj < 4; ++kj) {
        const int k = 4 * kb + kj;
        if (k >= bp) break;
        const int buf = kj & 1;
        // 1. the wave holding column k: candidates among rows not pivoted yet,
        //    maximum over the 16 owners (one DPP row of 16 lanes); the lane
        //    holding the pivot publishes its reciprocal with the key
        if ((tid >> 6) == (kb >> 2)) {
          u64 best = 0;
          double2 bv = make_double2(1.0, 0.0);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = 4 * rb + i;
            const double2 v = M[i][kj];
            if (owner) {
              S.pcol[buf][r] = v;
              if (r < bp && !((used >> r) & 1)) {
                const u64 key = pivot_key(fabs(v.x) + fabs(v.y), r);
                if (key > best) { best = key; bv = v; }
              }
            }
          }
          const u64 mine = best;
          best = umax64(best, dpp_u64<0xB1>(best));
          best = umax64(best, dpp_u64<0x4E>(best));
          best = umax64(best, dpp_u64<0x141>(best));
          best = umax64(best, dpp_u64<0x140>(best));
          if (owner && mine == best) {
            S.key[buf] = best;
            // zero pivot magnitude: the reciprocal of 1 keeps the elimination finite
            if (!((best >> kKeyBits) != 0)) bv = make_double2(1.0, 0.0);
            const double rd = 1.0 / (bv.x * bv.x + bv.y * bv.y);
            S.pinv[buf] = make_double2(bv.x * rd, -bv.y * rd);
          }
        }
        __syncthreads();
        // 2. every thread decodes the same pivot row p; its owners publish it
        const u64 gk = S.key[buf];
        const double2 inv = S.pinv[buf];
        double2 f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = cmul(S.pcol[buf][4 * rb + i], inv);
        int p = kKeyRows - 1 - int(gk & (kKeyRows - 1));
        if (p < 0 || p >= bp) p = k;   // (no candidate: cannot happen for k < bp)
        p = __builtin_amdgcn_readfirstlane(p);
        const double mag = __longlong_as_double((long long)(gk & ~(u64)(kKeyRows - 1)));
        if (!(mag > 0.0) || mag < thr) singular = true;
        const int pi = p & 3;
        const bool prow_owner = rb == (p >> 2);
        if (tid == 0) { S.prowi[k] = p; S.kinv[p] = k; }
        // the 16 threads of a column block are lanes 16 (cb % 4) .. + 15 of one
        // wave, so row p of this thread's columns comes from lane
        // 16 (cb % 4) + p / 4 of its own wave (pi is uniform: a scalar branch)
        double2 pr[4];
        {
          double2 sel[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) sel[j] = M[0][j];
#pragma unroll
          for (int i = 1; i < 4; ++i)
            if (pi == i)
#pragma unroll
              for (int j = 0; j < 4; ++j) sel[j] = M[i][j];
          const int src = ((16 * (cb & 3) + (p >> 2)) << 2);   // byte address of the source lane
#pragma unroll
          for (int j = 0; j < 4; ++j) pr[j] = bperm_d2(src, sel[j]);
        }
        // 3. M(i,j) -= f_i M(p,j) with f_i = M(i,k) / pivot for every row (row p
        //    and column k come out zero and are set next): column k <- -f,
        //    row p <- M(p,:) / pivot with 1 / pivot at column k
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) M[i][j] = cfms(M[i][j], f[i], pr[j]);
        if (owner) {
#pragma unroll
          for (int i = 0; i < 4; ++i) M[i][kj] = make_double2(-f[i].x, -f[i].y);
        }
        if (prow_owner) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (pi == i)
#pragma unroll
              for (int j = 0; j < 4; ++j) M[i][j] = (owner && j == kj) ? inv : cmul(pr[j], inv);
        }
        used |= (u64)1 << p;
      }
    }
    if (singular && tid == 0) a.status[e] = 1;
    __syncthreads();   // the last step's pivot labels
    // G(kinv[r], prowi[c]) = M(r, c): diag G and G(:, 0:rs) into LDS
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * rb + i, c = 4 * cb + j;
        if (r < bp && c < bp) {
          const int ga = S.kinv[r], gb = S.prowi[c];
          if (gb < rs) S.grs[gb][ga] = M[i][j];
          if (ga == gb) S.gd[ga] = M[i][j];
        }
      }
    __syncthreads();
    // outputs: four threads per node, partial sums over u = sub, sub + 4, ...
    const int sub = tid & 3;
    for (int q0 = 0; q0 < Lo.n_nodes; q0 += 64) {
      const int q = q0 + (tid >> 2);
      int l = 0, node = -1;
      if (q < Lo.n_nodes) {
        node = o.outnode[2 * (Lo.node_first + q)];
        l = o.outnode[2 * (Lo.node_first + q) + 1];
      }
      double re = 0.0, im = 0.0;
      if (node >= 0) {
        for (int u = sub; u < rs; u += 4) {
          double2 t = zero2();   // sum_v R(u, v) conj G(l, v)
          for (int v = 0; v < rs; ++v) {
            const double2 g = S.grs[v][l], rr = S.rs_[u][v];
            t.x += rr.x * g.x + rr.y * g.y;
            t.y += rr.y * g.x - rr.x * g.y;
          }
          const double2 gu = S.grs[u][l];
          re += gu.x * t.x - gu.y * t.y;
          im += gu.x * t.y + gu.y * t.x;
        }
      }
      re += dpp_f64<0xB1>(re); im += dpp_f64<0xB1>(im);
      re += dpp_f64<0x4E>(re); im += dpp_f64<0x4E>(im);
      if (node >= 0 && sub == 0) {
        o.diag_G[e * nn + node] = S.gd[l];
        o.diag_Gless[e * nn + node] = make_double2(re, im);
      }
    }
    __syncthreads();
  }
}

#ifndef FIND_TU
#error "kernels.hip is compiled once per kernel family: -DFIND_TU=1 .. 7"
#endif
// Launchers.  The source is compiled once per kernel family (FIND_TU = 1:
// k_stage with 1 panel row per thread, 2: with 2, 3: with 4 and 8, 4: k_final,
// 5: the one-wave form of k_stage, 6: its two-wave form) so that the families
// build in parallel.
#define FIND_LAUNCH_STAGE(R, T, C)                                                            \
  if (tc == T && cm == C) {                                                                   \
    hipLaunchKernelGGL((k_stage<R, T, C, kThreads, kThreads * R>), dim3(grid), dim3(kThreads), 0, st, a); \
    return hipGetLastError();                                                                 \
  }
// Solves with stencil-pattern scattering self-energies run the 32x32 wave
// tile with 4M products (or the eight-wave form) only.
#define FIND_LAUNCH_BONDS(R, NTH)                                                              \
  if (a.sbond) {                                                                              \
    if (tc != 0 || cm != 0) return hipErrorInvalidValue;                                      \
    hipLaunchKernelGGL((k_stage<R, 0, 0, NTH, NTH * R, true>), dim3(grid), dim3(NTH), 0, st, a); \
    return hipGetLastError();                                                                 \
  }
#if FIND_TU == 1 || FIND_TU == 2
hipError_t FIND_CAT(launch_stage_r, FIND_TU)(const StageArgs& a, int tc, int cm, int grid, hipStream_t st) {
  FIND_LAUNCH_BONDS(FIND_TU, kThreads)
  FIND_LAUNCH_STAGE(FIND_TU, 0, 0) FIND_LAUNCH_STAGE(FIND_TU, 1, 0) FIND_LAUNCH_STAGE(FIND_TU, 2, 0) FIND_LAUNCH_STAGE(FIND_TU, 3, 0)
  FIND_LAUNCH_STAGE(FIND_TU, 0, 1) FIND_LAUNCH_STAGE(FIND_TU, 1, 1) FIND_LAUNCH_STAGE(FIND_TU, 2, 1) FIND_LAUNCH_STAGE(FIND_TU, 3, 1)
  FIND_LAUNCH_STAGE(FIND_TU, kTileWg, 0) FIND_LAUNCH_STAGE(FIND_TU, kTileWg, 1)
  return hipErrorInvalidValue;
}
#endif
#if FIND_TU == 3
hipError_t launch_stage_r48(const StageArgs& a, int rpt, int tc, int cm, int grid, hipStream_t st) {
  if (rpt == 4) { FIND_LAUNCH_BONDS(4, kThreads) }
  if (rpt == 8) { FIND_LAUNCH_BONDS(8, kThreads) }
  if (rpt == 4) { FIND_LAUNCH_STAGE(4, 0, 0) FIND_LAUNCH_STAGE(4, 0, 1) }
  if (rpt == 8) { FIND_LAUNCH_STAGE(8, 0, 0) FIND_LAUNCH_STAGE(8, 0, 1) }
  return hipErrorInvalidValue;
}
#endif
#if FIND_TU == 5
// one wave per front (fronts of at most kWaveMaxFront nodes)
hipError_t launch_stage_w(const StageArgs& a, int rpt, int cm, int grid, hipStream_t st) {
  if (a.sbond) {
    if (cm != 0) return hipErrorInvalidValue;
    if (rpt == 1) { hipLaunchKernelGGL((k_stage<1, 0, 0, 64, kWaveMaxFront, true>), dim3(grid), dim3(64), 0, st, a); return hipGetLastError(); }
    if (rpt == 2) { hipLaunchKernelGGL((k_stage<2, 0, 0, 64, kWaveMaxFront, true>), dim3(grid), dim3(64), 0, st, a); return hipGetLastError(); }
    return hipErrorInvalidValue;
  }
#define FIND_LAUNCH_W(R, C)                                                                    \
  if (rpt == R && cm == C) {                                                                  \
    hipLaunchKernelGGL((k_stage<R, 0, C, 64, kWaveMaxFront>), dim3(grid), dim3(64), 0, st, a); \
    return hipGetLastError();                                                                 \
  }
  FIND_LAUNCH_W(1, 0) FIND_LAUNCH_W(2, 0) FIND_LAUNCH_W(1, 1) FIND_LAUNCH_W(2, 1)
#undef FIND_LAUNCH_W
  return hipErrorInvalidValue;
}
#endif
#if FIND_TU == 7
// eight waves per front (one workgroup per CU, 256 VGPRs per lane)
hipError_t launch_stage_w8(const StageArgs& a, int rpt, int cm, int grid, hipStream_t st) {
  const int tc = 0;   // (the eight-wave form has one wave tile)
  if (rpt == 1) { FIND_LAUNCH_BONDS(1, kEightWaveThreads) }
  if (rpt == 2) { FIND_LAUNCH_BONDS(2, kEightWaveThreads) }
  if (rpt == 4) { FIND_LAUNCH_BONDS(4, kEightWaveThreads) }
  if (rpt == 8) { FIND_LAUNCH_BONDS(8, kEightWaveThreads) }
#define FIND_LAUNCH_W8(R, C)                                                                   \
  if (rpt == R && cm == C) {                                                                  \
    hipLaunchKernelGGL((k_stage<R, 0, C, kEightWaveThreads, kEightWaveThreads * R>), dim3(grid), dim3(kEightWaveThreads), 0, st, a); \
    return hipGetLastError();                                                                 \
  }
  FIND_LAUNCH_W8(1, 0) FIND_LAUNCH_W8(2, 0) FIND_LAUNCH_W8(4, 0) FIND_LAUNCH_W8(8, 0)
  FIND_LAUNCH_W8(1, 1) FIND_LAUNCH_W8(2, 1) FIND_LAUNCH_W8(4, 1) FIND_LAUNCH_W8(8, 1)
#undef FIND_LAUNCH_W8
  return hipErrorInvalidValue;
}
#endif
#if FIND_TU == 6
// two waves per front (fronts of at most kTwoWaveMaxFront nodes)
hipError_t launch_stage_w2(const StageArgs& a, int rpt, int cm, int grid, hipStream_t st) {
  if (a.sbond) {
    if (cm != 0) return hipErrorInvalidValue;
    if (rpt == 1) { hipLaunchKernelGGL((k_stage<1, 0, 0, 128, kTwoWaveMaxFront, true>), dim3(grid), dim3(128), 0, st, a); return hipGetLastError(); }
    if (rpt == 2) { hipLaunchKernelGGL((k_stage<2, 0, 0, 128, kTwoWaveMaxFront, true>), dim3(grid), dim3(128), 0, st, a); return hipGetLastError(); }
    return hipErrorInvalidValue;
  }
#define FIND_LAUNCH_W2(R, C)                                                                   \
  if (rpt == R && cm == C) {                                                                  \
    hipLaunchKernelGGL((k_stage<R, 0, C, 128, kTwoWaveMaxFront>), dim3(grid), dim3(128), 0, st, a); \
    return hipGetLastError();                                                                 \
  }
  FIND_LAUNCH_W2(1, 0) FIND_LAUNCH_W2(2, 0) FIND_LAUNCH_W2(1, 1) FIND_LAUNCH_W2(2, 1)
#undef FIND_LAUNCH_W2
  return hipErrorInvalidValue;
}
#endif
#if FIND_TU == 4
hipError_t launch_final(const StageArgs& a, const OutArgs& o, int rpt, int grid, hipStream_t st) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_final<1, kThreads, kThreads * 1>), dim3(grid), dim3(kThreads), 0, st, a, o); break;
    case 2: hipLaunchKernelGGL((k_final<2, kThreads, kThreads * 2>), dim3(grid), dim3(kThreads), 0, st, a, o); break;
    case 4: hipLaunchKernelGGL((k_final<4, kThreads, kThreads * 4>), dim3(grid), dim3(kThreads), 0, st, a, o); break;
    case 8: hipLaunchKernelGGL((k_final<8, kThreads, kThreads * 8>), dim3(grid), dim3(kThreads), 0, st, a, o); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_final_w2(const StageArgs& a, const OutArgs& o, int rpt, int grid, hipStream_t st) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_final<1, 128, kTwoWaveMaxFront>), dim3(grid), dim3(128), 0, st, a, o); break;
    case 2: hipLaunchKernelGGL((k_final<2, 128, kTwoWaveMaxFront>), dim3(grid), dim3(128), 0, st, a, o); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_final_gj(const StageArgs& a, const OutArgs& o, int grid, hipStream_t st) {
  switch (a.sym) {
    case 0: hipLaunchKernelGGL((k_final_gj<256, 0>), dim3(grid), dim3(256), 0, st, a, o); break;
    case 1: hipLaunchKernelGGL((k_final_gj<256, 1>), dim3(grid), dim3(256), 0, st, a, o); break;
    case 3: hipLaunchKernelGGL((k_final_gj<256, 3>), dim3(grid), dim3(256), 0, st, a, o); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_final_w(const StageArgs& a, const OutArgs& o, int rpt, int grid, hipStream_t st) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_final<1, 64, kWaveMaxFront>), dim3(grid), dim3(64), 0, st, a, o); break;
    case 2: hipLaunchKernelGGL((k_final<2, 64, kWaveMaxFront>), dim3(grid), dim3(64), 0, st, a, o); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#endif
#undef FIND_LAUNCH_STAGE
#undef FIND_LAUNCH_BONDS

}  // namespace findmi
