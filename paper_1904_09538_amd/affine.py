"""Symbolic operation counting from a small affine loop-nest IR (the paper's
Section "Gathering Kernel Statistics": Algorithm opcount, per statement the
number of integer points of the loop domain projected onto the statement's
loops times the operations of one execution; Algorithm footcount, the
footprint of an array as the union of its accesses' index images).

A kernel's schedule is written as nested loops whose bounds are quasi-affine
in the problem parameters and the enclosing loop variables (integer-linear,
plus floor divisions by constants), with quasi-affine guards, and statements
that carry operation counts and array accesses.  Counting is then:

  * exact, by enumerating the domain (`count`, `footprint`), and
  * symbolic: the count of a parametric domain of this kind is a
    quasi-polynomial in the parameters (a polynomial whose coefficients
    depend on the parameters' residues modulo a period, on each chamber of
    the parameter space).  `quasi_polynomial` reconstructs it by exact
    rational interpolation from enumerated counts -- the period is the least
    common multiple of the floor divisors, the degree at most the loop depth
    -- and checks it on points it was not built from.  This interpolation
    approach to Ehrhart quasi-polynomials is Clauss's (1996); the paper uses
    Barvinok's algorithm through the barvinok library, which yields the
    same quasi-polynomials.

Granularities follow the paper: a statement's operations are per
execution; the kernels below enumerate lanes, waves or work-groups as loops
of the domain, so per-lane, per-wave or per-work-group counting is the choice
of which loops enclose the statement.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

# ---------------------------------------------------------------------- IR


@dataclass(frozen=True)
class Aff:
    """c0 + sum_k c_k x_k + sum_m d_m floor(a_m / q_m), x_k loop variables or
    parameters, a_m themselves Aff (quasi-affine expression)."""
    const: int = 0
    coef: Tuple[Tuple[str, int], ...] = ()
    floors: Tuple[Tuple["Aff", int, int], ...] = ()   # (inner, divisor q > 0, multiplier d)

    def ev(self, env: Dict[str, int]) -> int:
        v = self.const + sum(c * env[x] for x, c in self.coef)
        for inner, q, d in self.floors:
            v += d * (inner.ev(env) // q)
        return v

    def divisors(self) -> List[int]:
        out = []
        for inner, q, _ in self.floors:
            out.append(q)
            out += inner.divisors()
        return out

    # construction helpers
    def __add__(self, o):
        o = aff(o)
        coef: Dict[str, int] = dict(self.coef)
        for x, c in o.coef:
            coef[x] = coef.get(x, 0) + c
        return Aff(self.const + o.const, tuple(sorted((x, c) for x, c in coef.items() if c)),
                   self.floors + o.floors)

    __radd__ = __add__

    def __sub__(self, o):
        return self + aff(o) * -1

    def __rsub__(self, o):
        return aff(o) - self

    def __mul__(self, k: int):
        return Aff(self.const * k, tuple((x, c * k) for x, c in self.coef),
                   tuple((i, q, d * k) for i, q, d in self.floors))

    __rmul__ = __mul__

    def __floordiv__(self, q: int):
        return Aff(0, (), ((self, int(q), 1),))


def aff(x) -> Aff:
    if isinstance(x, Aff):
        return x
    if isinstance(x, int):
        return Aff(const=x)
    if isinstance(x, str):
        return Aff(coef=((x, 1),))
    raise TypeError(x)


def ceil_div(a, q: int) -> Aff:
    """ceil(a / q) = floor((a + q - 1) / q)."""
    return (aff(a) + (q - 1)) // q


@dataclass
class Access:
    array: str
    index: Tuple[Aff, ...]     # the index map I_{S,j}: loop variables -> array indices
    nbytes: int                # bytes per access (per executing lane)


@dataclass
class Stmt:
    """A statement: operations per execution (kind -> amount) and accesses."""
    name: str
    ops: Dict[str, int] = field(default_factory=dict)
    accesses: List[Access] = field(default_factory=list)


@dataclass
class Guard:
    """Statements inside run where lhs < rhs (affine), e.g. e < E."""
    lhs: Aff
    rhs: Aff
    body: List["Node"]


@dataclass
class Loop:
    """for var in [lo, hi): body."""
    var: str
    lo: Aff
    hi: Aff
    body: List["Node"]


Node = object   # Loop | Guard | Stmt


def loop(var, lo, hi, *body):
    return Loop(var, aff(lo), aff(hi), list(body))


def guard(lhs, rhs, *body):
    return Guard(aff(lhs), aff(rhs), list(body))


# ---------------------------------------------------------------------- exact counting

def _walk(nodes: Sequence[Node], env: Dict[str, int], visit):
    for nd in nodes:
        if isinstance(nd, Loop):
            lo, hi = nd.lo.ev(env), nd.hi.ev(env)
            for v in range(lo, hi):
                env[nd.var] = v
                _walk(nd.body, env, visit)
            env.pop(nd.var, None)
        elif isinstance(nd, Guard):
            if nd.lhs.ev(env) < nd.rhs.ev(env):
                _walk(nd.body, env, visit)
        else:
            visit(nd, env)


def _domain_size(nodes, env, stmt_name):
    """|pi_S(D)| for one statement: the number of points of the loop domain
    projected onto the loops enclosing S (guards included)."""
    n = [0]

    def visit(s, e):
        if s.name == stmt_name:
            n[0] += 1
    _walk(nodes, dict(env), visit)
    return n[0]


def count(kernel: Sequence[Node], params: Dict[str, int]) -> Dict[str, int]:
    """Algorithm opcount by enumeration: n_ops = sum_S |pi_S(D)| * n_ops,S, for
    every operation kind (bytes of each array access are kinds too:
    'bytes:<array>')."""
    stmts: Dict[str, Stmt] = {}

    def collect(nodes):
        for nd in nodes:
            if isinstance(nd, (Loop, Guard)):
                collect(nd.body)
            else:
                stmts[nd.name] = nd
    collect(kernel)
    totals: Dict[str, int] = {}
    for name, s in stmts.items():
        pts = _domain_size(kernel, params, name)
        for k, v in s.ops.items():
            totals[k] = totals.get(k, 0) + pts * v
        for a in s.accesses:
            key = "bytes:" + a.array
            totals[key] = totals.get(key, 0) + pts * a.nbytes
            key = "accesses:" + a.array
            totals[key] = totals.get(key, 0) + pts
    return totals


def footprint(kernel: Sequence[Node], params: Dict[str, int], array: str) -> int:
    """Algorithm footcount by enumeration: |F_v|, the number of distinct
    indices of `array` over the union of its accesses' images."""
    seen = set()

    def visit(s, env):
        for a in s.accesses:
            if a.array == array:
                seen.add(tuple(ix.ev(env) for ix in a.index))
    _walk(kernel, dict(params), visit)
    return len(seen)


def afr(kernel, params, array) -> Fraction:
    """Access-to-footprint ratio: element accesses / distinct elements accessed."""
    return Fraction(count(kernel, params).get("accesses:" + array, 0), footprint(kernel, params, array))


# ---------------------------------------------------------------------- quasi-polynomials

def _divisors_of(nodes) -> List[int]:
    out = []
    for nd in nodes:
        if isinstance(nd, Loop):
            out += nd.lo.divisors() + nd.hi.divisors() + _divisors_of(nd.body)
        elif isinstance(nd, Guard):
            out += nd.lhs.divisors() + nd.rhs.divisors() + _divisors_of(nd.body)
        else:
            for a in nd.accesses:
                for ix in a.index:
                    out += ix.divisors()
    return out


def _depth(nodes) -> int:
    d = 0
    for nd in nodes:
        if isinstance(nd, Loop):
            d = max(d, 1 + _depth(nd.body))
        elif isinstance(nd, Guard):
            d = max(d, _depth(nd.body))
    return d


@dataclass
class QuasiPolynomial:
    """sum over monomials prod_k p_k^{e_k} of coefficients that depend on the
    residues of the parameters modulo `period`; valid for every parameter
    value >= `start` (the chamber it was built on)."""
    params: Tuple[str, ...]
    period: int
    start: Tuple[int, ...]
    degree: int
    coeffs: Dict[Tuple[int, ...], Dict[Tuple[int, ...], Fraction]]   # residues -> monomial -> coeff

    def __call__(self, **vals) -> Fraction:
        x = tuple(vals[p] for p in self.params)
        r = tuple(v % self.period for v in x)
        return sum(c * math.prod(Fraction(v) ** e for v, e in zip(x, mono))
                   for mono, c in self.coeffs[r].items())

    def is_polynomial(self) -> bool:
        first = next(iter(self.coeffs.values()))
        return all(c == first for c in self.coeffs.values())

    def __str__(self):
        def one(cs):
            terms = []
            for mono, c in sorted(cs.items(), reverse=True):
                if c == 0:
                    continue
                m = "*".join(f"{p}^{e}" if e > 1 else p for p, e in zip(self.params, mono) if e)
                terms.append(f"{c}" + (f"*{m}" if m else ""))
            return " + ".join(terms) if terms else "0"
        if self.is_polynomial():
            return one(next(iter(self.coeffs.values())))
        return "; ".join(f"[{','.join(f'{p}%{self.period}={v}' for p, v in zip(self.params, r))}] {one(cs)}"
                         for r, cs in sorted(self.coeffs.items()))


def _monomials(nvars: int, degree: int):
    return [m for m in itertools.product(range(degree + 1), repeat=nvars) if sum(m) <= degree]


def _solve(rows: List[List[Fraction]], rhs: List[Fraction]) -> List[Fraction]:
    """Exact Gauss-Jordan elimination (square, nonsingular)."""
    n = len(rows)
    A = [r[:] + [b] for r, b in zip(rows, rhs)]
    for col in range(n):
        piv = next(i for i in range(col, n) if A[i][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        inv = 1 / A[col][col]
        A[col] = [v * inv for v in A[col]]
        for i in range(n):
            if i != col and A[i][col] != 0:
                f = A[i][col]
                A[i] = [a - f * b for a, b in zip(A[i], A[col])]
    return [A[i][n] for i in range(n)]


def quasi_polynomial(fn, params: Sequence[str], period: int, degree: int, start: Sequence[int],
                     checks: int = 2) -> QuasiPolynomial:
    """Reconstruct the quasi-polynomial f(params) from values fn(**params) on
    the chamber params >= start: per residue class modulo `period`, the
    polynomial of total degree <= `degree` through enough points of that
    class (a tensor grid of degree + 1 values per parameter, so the system
    is unisolvent), then `checks` further points per class must agree."""
    params = tuple(params)
    monos = _monomials(len(params), degree)
    coeffs = {}
    for res in itertools.product(range(period), repeat=len(params)):
        base = [s + ((r - s) % period) for s, r in zip(start, res)]
        grid = list(itertools.product(range(degree + 1), repeat=len(params)))
        pts = [tuple(b + period * k for b, k in zip(base, g)) for g in grid]
        # a unisolvent subset: the points whose grid multi-index has total degree <= degree
        pts = [p for p, g in zip(pts, grid) if sum(g) <= degree]
        A = [[Fraction(math.prod(Fraction(v) ** e for v, e in zip(p, m))) for m in monos] for p in pts]
        b = [Fraction(fn(**dict(zip(params, p)))) for p in pts]
        sol = _solve(A, b)
        cs = dict(zip(monos, sol))
        for c in range(checks):
            q = tuple(b_ + period * (degree + 1 + c + i) for i, b_ in enumerate(base))
            val = sum(cv * math.prod(Fraction(v) ** e for v, e in zip(q, m)) for m, cv in cs.items())
            if val != fn(**dict(zip(params, q))):
                raise ValueError(f"not a quasi-polynomial of degree {degree}, period {period} at {q}")
        coeffs[res] = cs
    return QuasiPolynomial(params, period, tuple(start), degree, coeffs)


def symbolic_count(kernel, op: str, params: Sequence[str], fixed: Dict[str, int], start: Sequence[int],
                   degree: int = None, period: int = None) -> QuasiPolynomial:
    """The count of operation kind `op` as a quasi-polynomial in `params`
    (other parameters fixed): period = lcm of the IR's floor divisors, degree
    = loop depth unless given."""
    if period is None:
        ds = _divisors_of(kernel)
        period = math.lcm(*ds) if ds else 1
    if degree is None:
        degree = _depth(kernel)
    return quasi_polynomial(lambda **v: count(kernel, {**fixed, **v}).get(op, 0), params, period, degree,
                            start)


# ---------------------------------------------------------------------- kernel schedules

def triangle():
    """The paper's worked example: the points (i, j) with p <= i < n and
    p <= j < i + 1."""
    return [loop("i", "p", "n", loop("j", "p", aff("i") + 1, Stmt("s", {"point": 1})))]


def stencil_vec(R: int):
    """The five-point stencil's vector path (n a multiple of 4, R rows per
    strip): work-group (bx, by) of 4 waves x 64 lanes; lane l of wave w owns
    columns j0 = (4 bx + w) 256 + 4 l (active while j0 < n); it loads u rows
    i_lo .. i_hi + 1 of its strip (i_hi = min(n, i_lo + R)) once each, 16
    bytes, plus the two right-halo values (8 bytes) when it is its wave's
    last lane or its right neighbour is past column n; it stores one 16-byte
    result per output row."""
    j0 = (4 * aff("bx") + aff("w")) * 256 + 4 * aff("l")
    i_lo = R * aff("by")

    def rows(r_end, i_end):
        # every lane computes its four results (five flops each); only the
        # active ones load and store
        return [loop("r", i_lo, r_end, guard(j0, "n",
                     Stmt("ld_u", {}, [Access("u", (aff("r"), j0), 16)]),
                     guard(62, aff("l"), Stmt("ld_halo63", {}, [Access("u", (aff("r"), j0 + 4), 8)])),
                     guard(aff("l"), 63, guard(aff("n") - 1, j0 + 4,
                                               Stmt("ld_halo_edge", {}, [Access("u", (aff("r"), j0 + 4), 8)]))))),
                loop("i", i_lo, i_end, Stmt("compute", {"flops": 20}),
                     guard(j0, "n", Stmt("st_res", {}, [Access("res", (aff("i"), j0), 16)])))]

    return [loop("by", 0, ceil_div("n", R), loop("bx", 0, ceil_div("n", 1024), loop("w", 0, 4, loop("l", 0, 64,
                 guard(i_lo + R, aff("n") + 1, *rows(i_lo + R + 2, i_lo + R)),     # a full strip
                 guard("n", i_lo + R, *rows(aff("n") + 2, "n"))))))]               # the last, short one


def stencil_reference():
    """The stencil as the paper states it: one statement per output point
    reading u at its five neighbours (for the footprint and AFR)."""
    i, j = aff("i"), aff("j")
    return [loop("i", 0, "n", loop("j", 0, "n", Stmt("s", {"flops": 5}, [
        Access("u", (i, j + 1), 4), Access("u", (i + 1, j), 4), Access("u", (i + 1, j + 1), 4),
        Access("u", (i + 1, j + 2), 4), Access("u", (i + 2, j + 1), 4), Access("res", (i, j), 4)])))]


def matmul_tiles():
    """The 128 x 128-tile matmul (n a multiple of 16): work-group (by, bx) of
    4 waves x 64 lanes, thread t = 64 w + l.  Per k-chunk of 16 the thread
    loads two 16-byte vectors of a row 128 by + t/2 (if below n) and one
    16-byte vector each at b columns 128 bx + 8 (t mod 16) and +4 (if below
    n); the four waves issue 64 matrix instructions (2048 flops each).
    Finally lane l of wave w stores, for i, j < 4, 16 bytes at row
    128 by + 64 (w / 2) + 16 i + (l mod 16) and column
    128 bx + 64 (w mod 2) + 16 j + 4 (l / 16) of c, where both are below n."""
    w, l = aff("w"), aff("l")
    lm16 = l - 16 * (l // 16)
    ar = 128 * aff("by") + 32 * w + (l // 2)
    bc = 128 * aff("bx") + 8 * lm16
    row = 128 * aff("by") + 64 * (w // 2) + 16 * aff("i") + lm16
    col = 128 * aff("bx") + 64 * (w - 2 * (w // 2)) + 16 * aff("j") + 4 * (l // 16)
    return [loop("by", 0, ceil_div("n", 128), loop("bx", 0, ceil_div("n", 128),
                 loop("kc", 0, ceil_div("n", 16),
                      loop("w", 0, 4,
                           Stmt("mfma", {"mfma_flops": 64 * 2048}),
                           loop("l", 0, 64,
                                guard(ar, "n", Stmt("ld_a", {}, [Access("a", (ar, 16 * aff("kc")), 32)])),
                                guard(bc, "n", Stmt("ld_b0", {}, [Access("b", (16 * aff("kc"), bc), 16)])),
                                guard(bc + 4, "n", Stmt("ld_b1", {}, [Access("b", (16 * aff("kc"), bc + 4), 16)]))))),
                 loop("w", 0, 4, loop("l", 0, 64, loop("i", 0, 4, guard(row, "n", loop("j", 0, 4,
                      guard(col, "n", Stmt("st_c", {}, [Access("c", (row, col), 16)])))))))))]


def dg_vec(nunit: int, kq: int, cb: int, ngroups: int, nmat: int = 3):
    """The DG forward's element loads, matrix work and output stores on the
    16-byte vector path without pipelined loads, over every wave-tile
    (parameter E; the tile streams only order the tiles): wave-tile q covers
    elements 16 cb q .. +16 cb; lane (c, g) of column block k loads the
    KQ/4 vectors of element e = 16 cb q + 16 k + c at nodes g KQ + 4 s below
    nunit, once per operator group (group 0 from memory, the others
    re-reading); each of the nmat * ceil(nunit/16) panels costs KQ cb
    matrix instructions (2048 flops) per wave-tile and a 16-byte store of
    nodes i0 + 4 g per lane whose element exists."""
    mblk = -(-nunit // 16)
    e = 16 * cb * aff("q") + 16 * aff("k") + aff("c")
    slab = aff("pp") // mblk
    node = 16 * (aff("pp") - mblk * slab) + 4 * aff("g")
    loads = [loop("s", 0, kq // 4,
                  guard(kq * aff("g") + 4 * aff("s"), nunit,
                        Stmt(f"ld_u{grp}", {}, [Access("u" if grp == 0 else "u_l2", (e,), 16)])))
             for grp in range(ngroups)]
    store = loop("pp", 0, nmat * mblk,
                 guard(node, nunit, Stmt("st_out", {}, [Access("out", (slab, e, node), 16)])))
    lane = loop("g", 0, 4, *loads, store)
    tile = [loop("pp", 0, nmat * mblk, Stmt("mfma", {"mfma_flops": kq * cb * 2048})),
            loop("k", 0, cb, loop("c", 0, 16, guard(e, "E", lane)))]
    return [loop("q", 0, ceil_div("E", 16 * cb), *tile)]
