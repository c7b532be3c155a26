// FIND elimination kernels for gfx950 (FP64 complex).
//
// One workgroup (256 threads, four wave64s) owns one (energy, elimination)
// work item at a time and walks a persistent loop over the stage's items.
// For an item with s eliminated and b kept nodes (n = s + b) it
//   1. assembles the front A_g (n x n) and Sigma_g (n x n) in [S ; B] order
//      from the stored U/R blocks of its sources and the original A / Sigma
//      (the block assembly of procedures updateBoundaryNodes and
//      updateAdjacentNodes; Sec. 3.1 for the Sigma blocks),
//   2. LU-factors the tall block [A(S,S); A(B,S)] with partial pivoting over
//      the S rows only (register-resident panels, MFMA trailing updates); the
//      B rows of the result hold L21 = A(B,S) U11^{-1},
//   3. forms L = A(B,S) A(S,S)^{-1} = L21 L11^{-1} P^T (eq. (express-L)),
//   4. computes [U | W] = [A(B,B) | Sigma(B,:)] - L [A(S,B) | Sigma(S,:)]
//      (eq. (major-update); W = [-L, I] Sigma), and
//   5. R = W(:,B) - W(:,S) L^dagger, which equals eq. (gless-update-rule)
//      Sigma(B,B) - L Sigma(S,B) - Sigma(B,S) L^dagger + L Sigma(S,S) L^dagger.
// The row permutation P is never applied to A(S,B) or Sigma: the products
// read row perm[k] for the k-th pivot instead.
// Complex products run on v_mfma_f64_16x16x4_f64 as four real products
// (re*re - im*im, re*im + im*re).
#include "kernels.hpp"

#include <climits>

namespace findmi {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cfms(double2 c, double2 a, double2 b) {  // c - a*b
  return make_double2(c.x - (a.x * b.x - a.y * b.y), c.y - (a.x * b.y + a.y * b.x));
}
__device__ __forceinline__ double2 cinv(double2 a) {
  double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }

// Entries of the original A = E I - H - Sigma_L - Sigma_R and of Sigma<.
struct Orig {
  const double* H;
  const double2* sig;
  const double2* sless;
  double2 E;
  int Nx, Ny, nst;

  __device__ double hval(int i, int j) const {
    const int xi = i % Nx, yi = i / Nx, xj = j % Nx, yj = j / Nx;
    const int dx = xj - xi, dy = yj - yi;
    const int plane = Nx * Ny;
    if (dy == 0) return dx == 1 ? H[plane + i] : dx == -1 ? H[plane + j] : 0.0;
    if (dx == 0) return dy == 1 ? H[2 * plane + i] : dy == -1 ? H[2 * plane + j] : 0.0;
    if (nst == 5) {
      if (dx == 1 && dy == 1) return H[3 * plane + i];
      if (dx == -1 && dy == -1) return H[3 * plane + j];
      if (dx == -1 && dy == 1) return H[4 * plane + yi * Nx + xj];  // i=(x+1,y), j=(x,y+1)
      if (dx == 1 && dy == -1) return H[4 * plane + yj * Nx + xi];  // i=(x,y+1), j=(x+1,y)
    }
    return 0.0;
  }
  __device__ double2 a(int i, int j) const {
    double2 v;
    if (i == j) v = make_double2(E.x - H[i], E.y);
    else v = make_double2(-hval(i, j), 0.0);
    const int yi = i / Nx, yj = j / Nx;
    if (yi == yj) {
      const int xi = i % Nx, xj = j % Nx;
      if (yi == 0) { double2 s = sig[xi * Nx + xj]; v.x -= s.x; v.y -= s.y; }
      if (yi == Ny - 1) { double2 s = sig[Nx * Nx + xi * Nx + xj]; v.x -= s.x; v.y -= s.y; }
    }
    return v;
  }
  __device__ double2 s(int i, int j) const {
    double2 v = zero2();
    const int yi = i / Nx, yj = j / Nx;
    if (yi == yj) {
      const int xi = i % Nx, xj = j % Nx;
      if (yi == 0) { double2 t = sless[xi * Nx + xj]; v.x += t.x; v.y += t.y; }
      if (yi == Ny - 1) { double2 t = sless[Nx * Nx + xi * Nx + xj]; v.x += t.x; v.y += t.y; }
    }
    return v;
  }
};

struct Lds {
  int node[kMaxFront];
  int srcpos[kMaxFront];
  int perm[kMaxFront];
  int ipiv[16];
  double2 rowP[16];
  double2 rowJ[16];
  double2 tri[16 * 16];
  double2 tinv[16 * 16];
  double2 tsq[16 * 16];
  double redv[4];
  int redi[4];
};

size_t stage_lds_bytes() { return sizeof(Lds); }

// C(M x N) <- Cinit - A(M x K) B(K x N), complex, one 32x32 tile per wave at a time.
template <class LA, class LB, class LC, class SC>
__device__ __forceinline__ void gemm_sub(int M, int N, int K, LA loadA, LB loadB, LC loadC, SC storeC) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tm = (M + 31) >> 5, tn = (N + 31) >> 5;
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = wave; t < tm * tn; t += 4) {
    const int r0 = (t % tm) << 5, c0 = (t / tm) << 5;
    d4 accR[2][2], accI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) { accR[i][j] = (d4){0, 0, 0, 0}; accI[i][j] = (d4){0, 0, 0, 0}; }
    for (int k = 0; k < K; k += 4) {
      const int kk = k + lk;
      double2 av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = r0 + 16 * i + lr;
        av[i] = (r < M && kk < K) ? loadA(r, kk) : zero2();
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = c0 + 16 * j + lr;
        bv[j] = (c < N && kk < K) ? loadB(kk, c) : zero2();
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].x, accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].y, accI[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[i].y, bv[j].y, accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].x, accI[i][j], 0, 0, 0);
        }
    }
    // D layout of the f64 16x16x4 MFMA: lane l, register q -> row 4q + l/16, column l%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = r0 + 16 * i + 4 * q + lk, c = c0 + 16 * j + lr;
          if (r < M && c < N) {
            double2 v = loadC(r, c);
            storeC(r, c, make_double2(v.x - accR[i][j][q], v.y - accI[i][j][q]));
          }
        }
  }
}

__device__ __forceinline__ void block_argmax(Lds& L, double& v, int& idx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  if (lane == 0) { L.redv[wave] = v; L.redi[wave] = idx; }
  __syncthreads();
  v = L.redv[0]; idx = L.redi[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    double ov = L.redv[w];
    int oi = L.redi[w];
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
}

// Inverse of the w x w unit-lower triangle held below the diagonal of L.tri
// (row-major, tri[i*16+j] = L_ij for i > j), written to L.tinv (zero outside
// w x w).  With L = I + N, N strictly lower and nilpotent,
// L^{-1} = (I - N)(I + N^2)(I + N^4)(I + N^8); 256 threads, one entry each.
__device__ void tri_inverse_unit_lower(Lds& L, int w) {
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  const double2 m = (i > j && i < w) ? make_double2(-L.tri[t].x, -L.tri[t].y) : zero2();
  __syncthreads();
  L.tsq[t] = m;
  L.tinv[t] = (i == j && i < w) ? make_double2(1.0 + m.x, m.y) : m;
  __syncthreads();
#pragma nounroll
  for (int step = 0; step < 3; ++step) {
    double2 a = zero2();
#pragma unroll 4
    for (int k = 0; k < 16; ++k) a = cfms(a, L.tsq[i * 16 + k], make_double2(-L.tsq[k * 16 + j].x, -L.tsq[k * 16 + j].y));
    __syncthreads();
    L.tsq[t] = a;            // M^(2^(step+1))
    __syncthreads();
    double2 p = L.tinv[t];   // P (I + A) = P + P A
#pragma unroll 4
    for (int k = 0; k < 16; ++k) p = cfms(p, L.tinv[i * 16 + k], make_double2(-L.tsq[k * 16 + j].x, -L.tsq[k * 16 + j].y));
    __syncthreads();
    L.tinv[t] = p;
    __syncthreads();
  }
}

// LU with partial pivoting (pivots searched among rows < s only) of the
// tall n x s block stored column-major (ld n) in FA.  perm[k] records which
// original row sits at position k.  Returns true if a zero pivot was met.
template <int RPT, int NB>
__device__ bool tall_lu(Lds& L, double2* FA, int n, int s) {
  const int tid = threadIdx.x;
  bool singular = false;
  for (int k0 = 0; k0 < s; k0 += NB) {
    const int kb = min(NB, s - k0);
    const int m = n - k0;          // panel rows
    const int ms = s - k0;         // pivot-eligible panel rows
    double2 P[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rho = tid + kThreads * q;
#pragma unroll
      for (int j = 0; j < NB; ++j)
        P[q][j] = (rho < m && j < kb) ? FA[(size_t)(k0 + j) * n + k0 + rho] : zero2();
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < kb) {
        double best = -1.0;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int rho = tid + kThreads * q;
          if (rho >= j && rho < ms) {
            double v = fabs(P[q][j].x) + fabs(P[q][j].y);
            if (v > best) { best = v; bi = rho; }
          }
        }
        block_argmax(L, best, bi);
        const int piv = bi;
        const int powner = piv % kThreads, pq = piv / kThreads;
        if (tid == powner) {
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            if (q == pq)
#pragma unroll
              for (int jj = 0; jj < NB; ++jj) L.rowP[jj] = P[q][jj];
        }
        if (tid == j) {
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) L.rowJ[jj] = P[0][jj];
        }
        if (tid == 0) L.ipiv[j] = k0 + piv;
        __syncthreads();
        if (piv != j) {
          if (tid == j) {
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) P[0][jj] = L.rowP[jj];
          }
          if (tid == powner) {
#pragma unroll
            for (int q = 0; q < RPT; ++q)
              if (q == pq)
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) P[q][jj] = L.rowJ[jj];
          }
        }
        double2 pv = L.rowP[j];
        if (!(best > 0.0)) { singular = true; pv = make_double2(1.0, 0.0); }
        const double2 inv = cinv(pv);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int rho = tid + kThreads * q;
          if (rho > j && rho < m) {
            const double2 l = cmul(P[q][j], inv);
            P[q][j] = l;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj)
              if (jj > j && jj < kb) P[q][jj] = cfms(P[q][jj], l, L.rowP[jj]);
          }
        }
        __syncthreads();
      }
    }
    // write the panel back; keep its unit-lower top block for the U12 solve
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rho = tid + kThreads * q;
      if (rho < m)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < kb) FA[(size_t)(k0 + j) * n + k0 + rho] = P[q][j];
    }
    if (tid < kb) {
#pragma unroll
      for (int j = 0; j < NB; ++j) L.tri[tid * 16 + j] = P[0][j];
    }
    if (tid == 0)
      for (int j = 0; j < kb; ++j) {
        const int r2 = L.ipiv[j];
        const int t = L.perm[k0 + j]; L.perm[k0 + j] = L.perm[r2]; L.perm[r2] = t;
      }
    __syncthreads();
    // apply this panel's row swaps to the other columns of the tall block
    for (int c = tid; c < s; c += kThreads) {
      if (c >= k0 && c < k0 + kb) continue;
      double2* col = FA + (size_t)c * n;
      for (int j = 0; j < kb; ++j) {
        const int r1 = k0 + j, r2 = L.ipiv[j];
        if (r1 != r2) { double2 t = col[r1]; col[r1] = col[r2]; col[r2] = t; }
      }
    }
    // U12 = L_panel^{-1} A12 for the columns right of the panel (in place)
    tri_inverse_unit_lower(L, kb);
    if (k0 + kb < s) {
      const int cb = k0 + kb;
      const Lds* LL = &L;
      gemm_sub(kb, s - cb, kb,
               [=](int r, int k) { double2 v = LL->tinv[r * 16 + k]; return make_double2(-v.x, -v.y); },
               [=](int k, int c) { return FA[(size_t)(cb + c) * n + k0 + k]; },
               [=](int r, int c) { return zero2(); },
               [=](int r, int c, double2 v) { FA[(size_t)(cb + c) * n + k0 + r] = v; });
    }
    __syncthreads();
    // trailing update of the tall block: rows k0+kb..n, columns k0+kb..s
    const int r0 = k0 + kb;
    if (r0 < s) {
      gemm_sub(n - r0, s - r0, kb,
               [=](int r, int k) { return FA[(size_t)(k0 + k) * n + r0 + r]; },
               [=](int k, int c) { return FA[(size_t)(r0 + c) * n + k0 + k]; },
               [=](int r, int c) { return FA[(size_t)(r0 + c) * n + r0 + r]; },
               [=](int r, int c, double2 v) { FA[(size_t)(r0 + c) * n + r0 + r] = v; });
    }
    __syncthreads();
  }
  return singular;
}

// X L11 = L21 in place (X -> FA rows s..n, columns 0..s); L11 unit lower.
__device__ void trsm_right_unit_lower(Lds& L, double2* FA, int n, int s, int b) {
  const int tid = threadIdx.x;
  const int nblk = (s + 15) / 16;
  for (int J = nblk - 1; J >= 0; --J) {
    const int j0 = 16 * J, j1 = min(s, j0 + 16), w = j1 - j0;
    if (j1 < s) {
      gemm_sub(b, w, s - j1,
               [=](int r, int k) { return FA[(size_t)(j1 + k) * n + s + r]; },
               [=](int k, int c) { return FA[(size_t)(j0 + c) * n + j1 + k]; },
               [=](int r, int c) { return FA[(size_t)(j0 + c) * n + s + r]; },
               [=](int r, int c, double2 v) { FA[(size_t)(j0 + c) * n + s + r] = v; });
    }
    {
      const int i = tid >> 4, jj = tid & 15;
      L.tri[tid] = (i < w && jj < w) ? FA[(size_t)(j0 + jj) * n + j0 + i] : zero2();
    }
    __syncthreads();
    tri_inverse_unit_lower(L, w);
    {
      const Lds* LL = &L;
      gemm_sub(b, w, w,
               [=](int r, int k) { return FA[(size_t)(j0 + k) * n + s + r]; },
               [=](int k, int c) { double2 v = LL->tinv[k * 16 + c]; return make_double2(-v.x, -v.y); },
               [=](int r, int c) { return zero2(); },
               [=](int r, int c, double2 v) { FA[(size_t)(j0 + c) * n + s + r] = v; });
    }
    __syncthreads();
  }
}

template <int RPT>
__global__ __launch_bounds__(kThreads) void k_stage(StageArgs a) {
  constexpr int NB = (32 / RPT) < 16 ? (32 / RPT) : 16;
  __shared__ Lds L;
  const int tid = threadIdx.x;
  const long long total = (long long)a.n_elims * a.nE;
  double2* FA = a.ws + (size_t)blockIdx.x * a.ws_stride;
  for (long long item = blockIdx.x; item < total; item += gridDim.x) {
    const int ei = int(item / a.nE), e = int(item % a.nE);
    const ElimDev E = a.elims[ei];
    const int s = E.s, b = E.b, n = E.n;
    double2* FS = FA + (size_t)n * n;
    double2* W = FS + (size_t)n * n;
    double2* pool = a.pool + (size_t)e * a.pool_stride;
    for (int k = tid; k < n; k += kThreads) {
      L.node[k] = a.map_node[E.map + k];
      L.srcpos[k] = a.map_srcpos[E.map + k];
    }
    for (int k = tid; k < s; k += kThreads) L.perm[k] = k;
    __syncthreads();
    // 1. assemble A_g and Sigma_g in [S ; B] order
    Orig o{a.H, a.sigma + (size_t)e * 2 * a.Nx * a.Nx, a.sless + (size_t)e * 2 * a.Nx * a.Nx,
           a.energies[e], a.Nx, a.Ny, a.nst};
    const double2* U0 = pool + E.src0;
    const double2* U1 = pool + E.src1;
    const size_t nn = (size_t)n * n;
    for (size_t idx = tid; idx < nn; idx += kThreads) {
      const int r = int(idx % n), c = int(idx / n);
      const int sr = L.srcpos[r] >> 24, sc = L.srcpos[c] >> 24;
      const int pr = L.srcpos[r] & 0xffffff, pc = L.srcpos[c] & 0xffffff;
      double2 av, sv;
      if (E.kind == 0) {
        if (sr == sc && sr == 0) {
          av = U0[(size_t)pc * E.ld0 + pr]; sv = U0[(size_t)E.ld0 * E.ld0 + (size_t)pc * E.ld0 + pr];
        } else if (sr == sc && sr == 1) {
          av = U1[(size_t)pc * E.ld1 + pr]; sv = U1[(size_t)E.ld1 * E.ld1 + (size_t)pc * E.ld1 + pr];
        } else {
          av = o.a(L.node[r], L.node[c]); sv = o.s(L.node[r], L.node[c]);
        }
      } else {  // final leaf block: [[U, I], [I, 0]] and [[R, 0], [0, 0]]
        if (sr == 0 && sc == 0) {
          av = U0[(size_t)pc * E.ld0 + pr]; sv = U0[(size_t)E.ld0 * E.ld0 + (size_t)pc * E.ld0 + pr];
        } else {
          av = make_double2((sr != sc && pr == pc) ? 1.0 : 0.0, 0.0); sv = zero2();
        }
      }
      FA[idx] = av;
      FS[idx] = sv;
    }
    __syncthreads();
    // 2. tall LU, 3. L = L21 L11^{-1}
    if (s > 0) {
      if (tall_lu<RPT, NB>(L, FA, n, s) && tid == 0) a.status[e] = 1;
      trsm_right_unit_lower(L, FA, n, s, b);
    }
    // 4. [U | W] = [A(B,B) | Sigma(B,:)] - L [A(perm,B) | Sigma(perm,:)]
    double2* Uo = pool + E.dst;
    double2* Ro = Uo + (size_t)b * b;
    const int* perm = L.perm;
    gemm_sub(b, b + n, s,
             [=](int r, int k) { return FA[(size_t)k * n + s + r]; },
             [=](int k, int c) {
               return c < b ? FA[(size_t)(s + c) * n + perm[k]] : FS[(size_t)(c - b) * n + perm[k]];
             },
             [=](int r, int c) { return c < b ? FA[(size_t)(s + c) * n + s + r] : FS[(size_t)(c - b) * n + s + r]; },
             [=](int r, int c, double2 v) {
               if (c < b) Uo[(size_t)c * b + r] = v; else W[(size_t)(c - b) * b + r] = v;
             });
    __syncthreads();
    // 5. R = W(:, B) - W(:, perm) L^dagger
    gemm_sub(b, b, s,
             [=](int r, int k) { return W[(size_t)perm[k] * b + r]; },
             [=](int k, int c) { return conjd(FA[(size_t)k * n + s + c]); },
             [=](int r, int c) { return W[(size_t)(s + c) * b + r]; },
             [=](int r, int c, double2 v) { Ro[(size_t)c * b + r] = v; });
    __syncthreads();
  }
}

// diag G = -U_final(l,l), diag G< = R_final(l,l); bond (i,j): G_ij, G<_ij and
// J = 2 Re(H_ij G<_ji), read from the final leaf blocks.
__global__ __launch_bounds__(64) void k_outputs(OutArgs a) {
  const int leaf = blockIdx.x, e = blockIdx.y;
  const LeafOutDev Lo = a.leaves[leaf];
  const long long dst = ((long long)Lo.elim_dst_hi << 32) | (unsigned)Lo.elim_dst_lo;
  const int bp = Lo.bprime;
  const double2* U = a.pool + (size_t)e * a.pool_stride + dst;
  const double2* R = U + (size_t)bp * bp;
  const size_t nn = (size_t)a.Nx * a.Ny;
  for (int k = threadIdx.x; k < Lo.n_nodes; k += blockDim.x) {
    const int node = a.outnode[2 * (Lo.node_first + k)];
    const int l = a.outnode[2 * (Lo.node_first + k) + 1];
    const double2 u = U[(size_t)l * bp + l];
    a.diag_G[e * nn + node] = make_double2(-u.x, -u.y);
    a.diag_Gless[e * nn + node] = R[(size_t)l * bp + l];
  }
  for (int k = threadIdx.x; k < Lo.n_bonds; k += blockDim.x) {
    const int* ob = a.outbond + 5 * (Lo.bond_first + k);
    const int bond = ob[0], li = ob[1], lj = ob[2], kk = ob[3], hf = ob[4];
    const size_t o = (size_t)e * a.n_bonds + bond;
    if (a.bond_G) { double2 u = U[(size_t)lj * bp + li]; a.bond_G[o] = make_double2(-u.x, -u.y); }
    if (a.bond_Gless) a.bond_Gless[o] = R[(size_t)lj * bp + li];
    if (a.bond_J) {
      const double h = a.H[(size_t)kk * nn + hf];
      a.bond_J[o] = 2.0 * h * R[(size_t)li * bp + lj].x;
    }
  }
}

hipError_t launch_stage(const StageArgs& a, int rpt, int grid, hipStream_t st) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL(k_stage<1>, dim3(grid), dim3(kThreads), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_stage<2>, dim3(grid), dim3(kThreads), 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_stage<4>, dim3(grid), dim3(kThreads), 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_stage<8>, dim3(grid), dim3(kThreads), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_outputs(const OutArgs& a, hipStream_t st) {
  if (a.n_leaves == 0 || a.nE == 0) return hipSuccess;
  hipLaunchKernelGGL(k_outputs, dim3(a.n_leaves, a.nE), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace findmi
