#!/usr/bin/env python3
"""Generator of the straight-line per-interface arithmetic of the HIP path.

Writes interface_gen.h next to this script.  The generated device functions
evaluate, for one Maxwellian at a time and in that Maxwellian's peculiar
frame (c = u - U, w = v - V), the velocity moments that the interface flux and
the interface point values need (Pan & Xu, arXiv:1412.4489, Sec. 2.2):

  * coef_*   -- the expansion coefficients a1, a2, A, d11, d12, d22, b1, b2,
                B of a Maxwellian from the derivatives of the conservative
                variables (the compatibility systems after eq. dis3), solved
                in closed form in the peculiar frame, where the Gram matrix
                <psi psi^T> is block diagonal;
  * mom_full_<term>, mom_half_<term>
             -- for one velocity polynomial X of eq. dis1 / eq. dis2 (a product
                of coefficient polynomials and particle velocities), the moments
                m0 = <psi' X> and (for flux terms) m1 = <c psi' X> over the whole
                velocity space (g0) or over the half space of one side (g_l on
                u > 0, g_r on u < 0).  The time weights are applied by the caller.

The moment functions are emitted in two stages: first the monomial
coefficients of the term's velocity polynomial (with shared subexpressions),
then the accumulation of every monomial's moments into the outputs, which
keeps only the coefficients live between the stages.

Whole-space central moments are closed forms in theta = 1/(2 lambda) and K;
half-space moments enter as the runtime table h[n] = <c^n>_half.  Products of
coefficient polynomials are formed symbolically, every moment that vanishes
by symmetry is dropped at generation time, and common subexpressions are
shared (sympy cse).  The leading terms (C1 g0 and C7 g_k) are evaluated
outside, in double precision.

Run:  python gen_interface.py   (needs sympy; the output is committed)
"""
import os
import sys

import sympy as sp
from sympy.printing.c import C99CodePrinter

HERE = os.path.dirname(os.path.abspath(__file__))

# ----------------------------------------------------------------------------
# polynomials in (c, w, z = xi^2) with sympy coefficients
# ----------------------------------------------------------------------------


class VP:
    __slots__ = ("t",)

    def __init__(self, t=None):
        self.t = {k: v for k, v in (t or {}).items() if v != 0}

    @staticmethod
    def const(x):
        return VP({(0, 0, 0): sp.sympify(x)})

    def __add__(self, o):
        if not isinstance(o, VP):
            o = VP.const(o)
        t = dict(self.t)
        for k, v in o.t.items():
            t[k] = t.get(k, 0) + v
        return VP(t)

    __radd__ = __add__

    def __neg__(self):
        return VP({k: -v for k, v in self.t.items()})

    def __sub__(self, o):
        return self + (-o)

    def __mul__(self, o):
        if not isinstance(o, VP):
            o = sp.sympify(o)
            return VP({k: v * o for k, v in self.t.items()})
        t = {}
        for k1, v1 in self.t.items():
            for k2, v2 in o.t.items():
                k = (k1[0] + k2[0], k1[1] + k2[1], k1[2] + k2[2])
                t[k] = t.get(k, 0) + v1 * v2
        return VP(t)

    __rmul__ = __mul__


C = VP({(1, 0, 0): 1})
Wv = VP({(0, 1, 0): 1})
Z = VP({(0, 0, 1): 1})
ZETA = (C * C + Wv * Wv + Z) * sp.Rational(1, 2)  # (c^2 + w^2 + xi^2) / 2


def lin(a, dim):
    """a0 + a1 c + a2 w + a3 zeta (2D) ; a0 + a1 c + a2 zeta (1D), peculiar frame"""
    if dim == 2:
        return VP.const(a[0]) + C * a[1] + Wv * a[2] + ZETA * a[3]
    z1 = (C * C + Z) * sp.Rational(1, 2)
    return VP.const(a[0]) + C * a[1] + z1 * a[2]


def psi(dim):
    if dim == 2:
        return [VP.const(1), C, Wv, ZETA]
    return [VP.const(1), C, (C * C + Z) * sp.Rational(1, 2)]


def dfact(n):  # (n-1)!! for even n: <s^n> = (n-1)!! theta^(n/2)
    r = 1
    for k in range(n - 1, 0, -2):
        r *= k
    return r


class Moments:
    """Moment functional of one Maxwellian in its peculiar frame."""

    def __init__(self, dim, half, TH, KP, H=None):
        self.dim, self.half, self.TH, self.KP, self.H = dim, half, TH, KP, H

    def mono(self, a, b, e):
        if self.dim == 1 and b:
            return 0
        if b % 2:
            return 0
        if not self.half and a % 2:
            return 0
        if self.half:
            return self.H[a] * dfact(b) * self.KP[e] * self.TH[b // 2 + e]
        return dfact(a) * dfact(b) * self.KP[e] * self.TH[(a + b) // 2 + e]

    def of(self, P):
        s = 0
        for (a, b, e), v in P.t.items():
            m = self.mono(a, b, e)
            if m != 0:
                s += v * m
        return s

    def psi(self, P, extra=None):
        """< psi'_i P > (or < extra psi'_i P >)"""
        if extra is not None:
            P = P * extra
        return [self.of(P * p) for p in psi(self.dim)]


# ----------------------------------------------------------------------------
# code emission
# ----------------------------------------------------------------------------


class Printer(C99CodePrinter):
    def _print_Rational(self, e):
        return "T(%s)" % repr(float(e.p) / float(e.q))

    def _print_Integer(self, e):
        return "T(%d)" % int(e)

    def _print_Float(self, e):
        return "T(%s)" % repr(float(e))

    def _print_Pow(self, e):
        b, x = e.args
        if x.is_Integer and 2 <= int(x) <= 4:
            s = self._print(b)
            return "(" + "*".join([s] * int(x)) + ")"
        if x == -1:
            return "(T(1)/%s)" % self._print(b)
        return super()._print_Pow(e)


PR = Printer()


def emit(assign, outputs, indent="  "):
    """assign: list of (name, expr) final outputs; cse and print."""
    names = [n for n, _ in outputs]
    exprs = [sp.sympify(e) for _, e in outputs]
    repl, red = sp.cse(exprs, symbols=sp.numbered_symbols("t_"), optimizations="basic")
    lines = []
    for s, e in repl:
        lines.append(f"{indent}const T {s} = {PR.doprint(e)};")
    for n, e in zip(names, red):
        lines.append(f"{indent}{n} = {PR.doprint(e)};")
    nops = sum(sp.count_ops(e) for _, e in repl) + sum(sp.count_ops(e) for e in red)
    return lines, nops


# ----------------------------------------------------------------------------
# the physics
# ----------------------------------------------------------------------------


def symvec(name, n):
    return [sp.Symbol(f"{name}[{i}]") for i in range(n)]


def theta_syms():
    TH = [sp.Integer(1)] + [sp.Symbol(f"th[{k}]") for k in range(1, 8)]  # th[k] = theta^k
    KP = [sp.Integer(1)] + [sp.Symbol(f"kp[{k}]") for k in range(1, 5)]  # K(K+2)...
    return TH, KP


def solve_peculiar(b, dim, TH, N):
    """closed-form solve of <a psi'> = b with the Gram matrix of the peculiar
    frame: only (1, zeta) couple.  N = total thermal degrees of freedom."""
    th = TH[1]
    if dim == 2:
        z1 = N * th / 2
        det = N * th * th / 2
        a3 = (b[3] - z1 * b[0]) / det
        return [b[0] - z1 * a3, b[1] / th, b[2] / th, a3]
    z1 = N * th / 2
    det = N * th * th / 2
    a2 = (b[2] - z1 * b[0]) / det
    return [b[0] - z1 * a2, b[1] / th, a2]


def gen_coefficients(dim, which):
    """Stages of the coefficient computation for one Maxwellian.
    which: 0 = g0 (all nine), 1 = side Euler, 2 = side NS."""
    nv = dim + 2
    TH, KP = theta_syms()
    Nsym = sp.Symbol("nthermal")
    M = Moments(dim, False, TH, KP)
    Us, Vs = sp.Symbol("U"), sp.Symbol("V")
    bx, by, bxx, bxy, byy = (symvec(n, nv) for n in ("bx", "by", "bxx", "bxy", "byy"))
    stages = []

    def solve(b):
        return solve_peculiar(b, dim, TH, Nsym)

    # stage 1: a1, a2
    ax = solve(bx)
    out = [(f"ax[{i}]", ax[i]) for i in range(nv)]
    if dim == 2:
        ay = solve(by)
        out += [(f"ay[{i}]", ay[i]) for i in range(nv)]
    stages.append(out)
    AX = lin(symvec("ax", nv), dim)
    AY = lin(symvec("ay", nv), dim) if dim == 2 else VP()
    u = C + Us
    v = Wv + Vs
    # stage 2: d11, d12, d22 (and A)
    out = []
    m = M.psi(AX * AX)
    dxx = solve([bxx[i] - m[i] for i in range(nv)])
    out += [(f"dxx[{i}]", dxx[i]) for i in range(nv)]
    if dim == 2:
        m = M.psi(AX * AY)
        dxy = solve([bxy[i] - m[i] for i in range(nv)])
        out += [(f"dxy[{i}]", dxy[i]) for i in range(nv)]
        m = M.psi(AY * AY)
        dyy = solve([byy[i] - m[i] for i in range(nv)])
        out += [(f"dyy[{i}]", dyy[i]) for i in range(nv)]
    if which != 1:
        m = M.psi(AX * u + AY * v)
        A = solve([-m[i] for i in range(nv)])
        out += [(f"At[{i}]", A[i]) for i in range(nv)]
    stages.append(out)
    if which == 1:
        return stages
    AT = lin(symvec("At", nv), dim)
    DXX = AX * AX + lin(symvec("dxx", nv), dim)
    DXY = AX * AY + lin(symvec("dxy", nv), dim) if dim == 2 else VP()
    DYY = AY * AY + lin(symvec("dyy", nv), dim) if dim == 2 else VP()
    out = []
    m = M.psi(DXX * u + DXY * v + AT * AX)
    b1 = solve([-m[i] for i in range(nv)])
    out += [(f"bxt[{i}]", b1[i]) for i in range(nv)]
    if dim == 2:
        m = M.psi(DXY * u + DYY * v + AT * AY)
        b2 = solve([-m[i] for i in range(nv)])
        out += [(f"byt[{i}]", b2[i]) for i in range(nv)]
    stages.append(out)
    if which == 2:
        return stages
    TX = AT * AX + lin(symvec("bxt", nv), dim)
    TY = AT * AY + lin(symvec("byt", nv), dim) if dim == 2 else VP()
    m = M.psi(TX * u + TY * v + AT * AT)
    B = solve([-m[i] for i in range(nv)])
    stages.append([(f"Bt[{i}]", B[i]) for i in range(nv)])
    return stages


def coefficient_polys(dim, viscous_side, role):
    nv = dim + 2
    AX = lin(symvec("ax", nv), dim)
    AY = lin(symvec("ay", nv), dim) if dim == 2 else VP()
    AT = lin(symvec("At", nv), dim)
    D11 = lin(symvec("dxx", nv), dim)
    D12 = lin(symvec("dxy", nv), dim) if dim == 2 else VP()
    D22 = lin(symvec("dyy", nv), dim) if dim == 2 else VP()
    B1 = lin(symvec("bxt", nv), dim)
    B2 = lin(symvec("byt", nv), dim) if dim == 2 else VP()
    BT = lin(symvec("Bt", nv), dim)
    P = dict(AX=AX, AY=AY, AT=AT)
    P["DXX"] = AX * AX + D11
    P["DXY"] = AX * AY + D12
    P["DYY"] = AY * AY + D22
    if role == "hydro" or viscous_side:
        P["TX"] = AT * AX + B1
        P["TY"] = AT * AY + B2
    if role == "hydro":
        P["TTT"] = AT * AT + BT
    return P


# terms of the interface distribution: name -> (velocity polynomial builder,
# coefficient vectors it reads, whether its flux moment <c psi' X> is needed)
def term_polys(dim):
    nv = dim + 2
    U, V = sp.Symbol("U"), sp.Symbol("V")
    u, v = C + U, Wv + V
    vec = {n: lin(symvec(n, nv), dim) for n in ("ax", "ay", "At", "dxx", "dxy", "dyy", "bxt", "byt", "Bt")}
    if dim == 1:
        for n in ("ay", "dxy", "dyy", "byt"):
            vec[n] = VP()
    AX, AY, AT = vec["ax"], vec["ay"], vec["At"]
    DXX = AX * AX + vec["dxx"]
    DXY = AX * AY + vec["dxy"]
    DYY = AY * AY + vec["dyy"]
    TX = AT * AX + vec["bxt"]
    TY = AT * AY + vec["byt"]
    TTT = AT * AT + vec["Bt"]
    T = {
        # term       polynomial                                   inputs                     flux
        "conv": (AX * u + AY * v, ["ax", "ay"], True),
        "A": (AT, ["At"], True),
        "quad": (DXX * u * u + DXY * u * v * 2 + DYY * v * v, ["ax", "ay", "dxx", "dxy", "dyy"], True),
        "ttt": (TTT, ["At", "Bt"], True),
        "tlin": (TX * u + TY * v, ["ax", "ay", "At", "bxt", "byt"], True),
        "dyy": (DYY, ["ay", "dyy"], True),
        "ay": (AY, ["ay"], False),
        "inner": (DXY * u + DYY * v, ["ax", "ay", "dxy", "dyy"], False),
        "ty": (TY, ["ay", "At", "byt"], False),
    }
    if dim == 1:
        for n in ("dyy", "ay", "inner", "ty"):
            del T[n]
    return T


def gen_term(dim, name, half):
    TH, KP = theta_syms()
    H = [sp.Symbol(f"h[{n}]") for n in range(12)] if half else None
    M = Moments(dim, half, TH, KP, H)
    P, ins, flux = term_polys(dim)[name]
    out = [(f"m0[{i}]", e) for i, e in enumerate(M.psi(P))]
    if flux:
        out += [(f"m1[{i}]", e) for i, e in enumerate(M.psi(P, C))]
    return ins, flux, out


def gen_term_two_stage(dim, name, half):
    """The same moments as gen_term in two stages with separate common
    subexpressions: (1) the monomial coefficients p_abe of the term's velocity
    polynomial X = sum p_abe c^a w^b z^e from the expansion coefficients;
    (2) m0_i = sum p_abe <psi'_i c^a w^b z^e>, m1_i = sum p_abe <c psi'_i ...>.
    Only the coefficients are live between the stages (a smaller register
    peak than one expanded expression per output)."""
    TH, KP = theta_syms()
    H = [sp.Symbol(f"h[{n}]") for n in range(12)] if half else None
    M = Moments(dim, half, TH, KP, H)
    P, ins, flux = term_polys(dim)[name]
    keys = sorted(P.t)
    psyms = {k: sp.Symbol(f"p_{k[0]}_{k[1]}_{k[2]}") for k in keys}
    stage1 = [(str(psyms[k]), P.t[k]) for k in keys]
    # stage 2 as accumulation, monomial by monomial: out += p_k * <psi' mono_k>
    outs = [f"m0[{i}]" for i in range(len(psi(dim)))]
    if flux:
        outs += [f"m1[{i}]" for i in range(len(psi(dim)))]
    acc = []
    for k in keys:
        mono = VP({k: 1})
        vals = M.psi(mono) + (M.psi(mono, C) if flux else [])
        for o, v in zip(outs, vals):
            v = sp.expand(v)
            if v != 0:
                acc.append((o, psyms[k], v))
    return ins, flux, stage1, (outs, acc)


HEADER = """// interface_gen.h -- GENERATED by gen_interface.py; do not edit by hand.
//
// Straight-line velocity-moment arithmetic of one Maxwellian in its peculiar
// frame (c = u - U, w = v - V) for the interface evaluation of the compact
// third-order gas-kinetic scheme (Pan & Xu, arXiv:1412.4489, Sec. 2.2):
// expansion coefficients from the compatibility systems, and the moments of
// eq. dis1 (hydrodynamic part, whole space) and eq. dis2 (kinetic part, half
// space) without their leading terms.  th[k] = theta^k with theta = 1/(2
// lambda); kp[e] = K (K+2) ... (K+2e-2); h[n] = <c^n> over the half space.
#pragma once
"""


# terms generated in two stages (see gen_term_two_stage)
TWO_STAGE = ("conv", "A", "quad", "ttt", "tlin", "dyy", "ay", "inner", "ty")


def main():
    body = [HEADER]
    report = []
    emitted = []
    for dim in (2, 1):
        nv = dim + 2
        for which, tag in ((0, "g0"), (1, "side_euler"), (2, "side_ns")):
            stages = gen_coefficients(dim, which)
            sig = (f"template <typename T>\n__device__ __forceinline__ void coef_{tag}_{dim}d(\n"
                   f"    const T* __restrict__ th, const T* __restrict__ kp, T nthermal, T U, T V,\n"
                   f"    const T* bx, const T* by, const T* bxx, const T* bxy, const T* byy,\n"
                   f"    T* ax, T* ay, T* At, T* dxx, T* dxy, T* dyy, T* bxt, T* byt, T* Bt) {{")
            lines = [sig]
            total = 0
            for st in stages:  # one block per stage: the outputs of a stage feed the next
                l, n = emit(None, st, indent="    ")
                lines += ["  {"] + l + ["  }"]
                total += n
            lines.append("}\n")
            body += lines
            report.append((f"coef_{tag}_{dim}d", total))
        for half, tag in ((False, "full"), (True, "half")):
            for name in term_polys(dim):
                if half and name in ("ttt",):
                    continue  # B is not part of the kinetic part
                if name in TWO_STAGE:
                    ins, flux, stage1, (onames, acc) = gen_term_two_stage(dim, name, half)
                    l1, n1 = emit(None, stage1, indent="    ")
                    decl = "  T " + ", ".join(n for n, _ in stage1) + ";"
                    l2 = [f"  {o} = T(0);" for o in onames]
                    n2 = 0
                    for o, pk, v in acc:
                        l2.append(f"  {o} += {pk} * ({PR.doprint(v)});")
                        n2 += 2 + sp.count_ops(v)
                    l = [decl, "  {"] + l1 + ["  }"] + l2
                    # the algorithmic count: the same moments as one expanded
                    # expression per output with shared subexpressions
                    _, _, outs_cse = gen_term(dim, name, half)
                    _, n = emit(None, outs_cse)
                    emitted.append((f"mom_{tag}_{name}_{dim}d", n1 + n2))
                else:
                    ins, flux, outs = gen_term(dim, name, half)
                    l, n = emit(None, outs)
                args = ", ".join(f"const T* {a}" for a in ins)
                hh = "const T* __restrict__ h, " if half else ""
                res = "T* m0, T* m1" if flux else "T* m0"
                body.append(f"template <typename T>\n__device__ __forceinline__ void mom_{tag}_{name}_{dim}d(\n"
                            f"    const T* __restrict__ th, const T* __restrict__ kp, {hh}T U, T V, {args},\n"
                            f"    {res}) {{")
                body += l
                body.append("}\n")
                report.append((f"mom_{tag}_{name}_{dim}d", n))
    out = os.path.join(HERE, "interface_gen.h")
    with open(out, "w") as f:
        f.write("\n".join(body))
    em = dict(emitted)
    for name, n in report:
        print(f"{name:24s} ~{n} ops" + (f"   (emitted form ~{em[name]})" if name in em else ""))
    # floating-point operations (sympy count_ops: one per +, -, *, /) of the
    # generated functions in the form with shared subexpressions (the emitted
    # two-stage form trades some of them for a lower register peak), used as
    # the algorithmic count of an interface
    import json
    with open(os.path.join(HERE, "interface_ops.json"), "w") as f:
        json.dump({name: int(n) for name, n in report}, f, indent=1)


if __name__ == "__main__":
    sys.setrecursionlimit(100000)
    main()
