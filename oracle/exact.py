"""Exact brute force on tiny meshes (pure Python, Gaussian rationals).

Every float input (H values, Sigma, Sigma<, E) is converted to the exact
rational it represents, A is assembled by enumerating all node pairs (a
construction separate from ``dense``), inverted by exact Gauss-Jordan
elimination, and G< = G Sigma< G^dagger is formed exactly.  The float
oracles must agree with this to ~1e-13 relative; it pins the definition of
A (signs, contact placement, stencil orientation), of G<, and of the bond
outputs.  Only for n = Nx*Ny <= ~16.
"""
from __future__ import annotations

from fractions import Fraction


class Q:
    """Exact complex rational re + i*im."""
    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = re if isinstance(re, Fraction) else Fraction(re)
        self.im = im if isinstance(im, Fraction) else Fraction(im)

    @staticmethod
    def of(z) -> "Q":
        z = complex(z)
        return Q(Fraction(z.real), Fraction(z.imag))

    def __add__(self, o): return Q(self.re + o.re, self.im + o.im)
    def __sub__(self, o): return Q(self.re - o.re, self.im - o.im)
    def __neg__(self): return Q(-self.re, -self.im)
    def __mul__(self, o): return Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)
    def conj(self): return Q(self.re, -self.im)
    def is_zero(self): return self.re == 0 and self.im == 0

    def inv(self):
        d = self.re * self.re + self.im * self.im
        return Q(self.re / d, -self.im / d)

    def __complex__(self): return complex(float(self.re), float(self.im))


ZERO = Q(0, 0)


def coords(i: int, Nx: int):
    return i % Nx, i // Nx


def h_value(H, Nx: int, Ny: int, i: int, j: int) -> Fraction:
    """H_ij by looking at the displacement between the two nodes."""
    xi, yi = coords(i, Nx)
    xj, yj = coords(j, Nx)
    dx, dy = xj - xi, yj - yi
    nst = len(H)
    if dx == 0 and dy == 0:
        return Fraction(float(H[0][yi][xi]))
    if (dx, dy) == (1, 0):
        return Fraction(float(H[1][yi][xi]))
    if (dx, dy) == (-1, 0):
        return Fraction(float(H[1][yj][xj]))
    if (dx, dy) == (0, 1):
        return Fraction(float(H[2][yi][xi]))
    if (dx, dy) == (0, -1):
        return Fraction(float(H[2][yj][xj]))
    if nst == 5:
        if (dx, dy) == (1, 1):
            return Fraction(float(H[3][yi][xi]))
        if (dx, dy) == (-1, -1):
            return Fraction(float(H[3][yj][xj]))
        if (dx, dy) == (-1, 1):   # i = (x+1, y), j = (x, y+1) with x = xj
            return Fraction(float(H[4][yi][xj]))
        if (dx, dy) == (1, -1):   # i = (x, y+1), j = (x+1, y) with x = xi
            return Fraction(float(H[4][yj][xi]))
    return Fraction(0)


def bond_sigma_value(B, Nx: int, Ny: int, i: int, j: int) -> Q:
    """Entry (i, j) of a stencil-pattern self-energy given per bond plane with
    two values per bond (index 0: from the bond's first node to its second,
    index 1: back), found from the displacement between the two nodes."""
    if B is None:
        return Q()
    xi, yi = coords(i, Nx)
    xj, yj = coords(j, Nx)
    dx, dy = xj - xi, yj - yi
    nb = len(B)
    if (dx, dy) == (1, 0):
        return Q.of(B[0][yi][xi][0])
    if (dx, dy) == (-1, 0):
        return Q.of(B[0][yj][xj][1])
    if (dx, dy) == (0, 1):
        return Q.of(B[1][yi][xi][0])
    if (dx, dy) == (0, -1):
        return Q.of(B[1][yj][xj][1])
    if nb == 4:
        if (dx, dy) == (1, 1):
            return Q.of(B[2][yi][xi][0])
        if (dx, dy) == (-1, -1):
            return Q.of(B[2][yj][xj][1])
        if (dx, dy) == (-1, 1):   # first node i = (x+1, y), second j = (x, y+1), x = xj
            return Q.of(B[3][yi][xj][0])
        if (dx, dy) == (1, -1):   # i = (x, y+1) is the second node, j = (x+1, y) the first, x = xi
            return Q.of(B[3][yj][xi][1])
    return Q()


def contact_value(S, Nx: int, Ny: int, i: int, j: int) -> Q:
    """Entry (i, j) of the dense contact matrix: S[c][xi][xj] when both nodes
    sit on contact column c (left y = 0, right y = Ny-1)."""
    xi, yi = coords(i, Nx)
    xj, yj = coords(j, Nx)
    v = Q()
    if yi == 0 and yj == 0:
        v = v + Q.of(S[0][xi][xj])
    if yi == Ny - 1 and yj == Ny - 1:
        v = v + Q.of(S[1][xi][xj])
    return v


def exact_inverse(M):
    n = len(M)
    A = [row[:] + [Q(1 if r == c else 0) for c in range(n)] for r, row in enumerate(M)]
    for col in range(n):
        piv = next(r for r in range(col, n) if not A[r][col].is_zero())
        A[col], A[piv] = A[piv], A[col]
        inv = A[col][col].inv()
        A[col] = [v * inv for v in A[col]]
        for r in range(n):
            if r != col and not A[r][col].is_zero():
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return [row[n:] for row in A]


def exact_solve(Nx: int, Ny: int, H, E, sigma_e, sless_e, bond_pairs, sb_e=None, slb_e=None):
    """Exact diag G, diag G<, and (G_ij, G<_ij, J) for each (i, j) in
    ``bond_pairs`` at one energy, with the stencil-pattern self-energies
    sb_e, slb_e ([nst-1][Ny][Nx][2]) when given.  Returns python complex /
    float values."""
    n = Nx * Ny
    Eq = Q.of(E)
    A = [[ZERO] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            v = (Q(-h_value(H, Nx, Ny, i, j), 0) - contact_value(sigma_e, Nx, Ny, i, j)
                 - bond_sigma_value(sb_e, Nx, Ny, i, j))
            if i == j:
                v = v + Eq
            A[i][j] = v
    G = exact_inverse(A)
    S = [[contact_value(sless_e, Nx, Ny, i, j) + bond_sigma_value(slb_e, Nx, Ny, i, j) for j in range(n)]
         for i in range(n)]

    def gless(a, b):
        acc = Q()
        for k in range(n):
            if G[a][k].is_zero():
                continue
            for m in range(n):
                if S[k][m].is_zero():
                    continue
                acc = acc + G[a][k] * S[k][m] * G[b][m].conj()
        return acc

    diag_G = [complex(G[i][i]) for i in range(n)]
    diag_Gl = [complex(gless(i, i)) for i in range(n)]
    bonds = []
    for (i, j) in bond_pairs:
        h = h_value(H, Nx, Ny, i, j)
        glji = gless(j, i)
        J = 2 * (h * glji.re)
        bonds.append((complex(G[i][j]), complex(gless(i, j)), float(J)))
    return diag_G, diag_Gl, bonds
