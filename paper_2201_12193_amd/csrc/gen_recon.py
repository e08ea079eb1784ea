#!/usr/bin/env python3
"""Generate recon_gen.h: the linear parts of the HWENO reconstruction.

Derived here with exact rational arithmetic (sympy) from the moment
conditions of the paper:
  * 1D q_2, q_3, q_4 (eq. q): square systems on the cells i-1, i, i+1.
  * 2D q_2, q_3, q_4 (eqs. 2D-q2 .. 2D-q4): the centre cell average is kept
    exactly and every other condition is fitted in the unweighted
    least-squares sense (KKT system, solved exactly).
  * smoothness-indicator quadratic forms of eq. (beta) / (2D-beta) in the
    cell's reference coordinates (kappa = 2, 3, 5; every multi-index once).
  * evaluation of a polynomial at the Gauss-Lobatto points of eq. (F)
    (nodes +-1/2, +-sqrt(5)/10; tensor grid in 2D).
  * the first-moment modification of eq. (p0)/(vi).

The 2D stencil is symmetric under x -> -x and y -> -y, so the maps
decouple by the parity class (a mod 2, b mod 2) of the monomial xi^a eta^b
once the stencil data are combined into even/odd sums and differences.  The
generator applies that change of variables exactly and emits only the
non-zero entries, which roughly halves the arithmetic.

Output: straight-line FP64 device code with each constant written as an
exact hexadecimal literal of the correctly rounded double.

Run:  python gen_recon.py > recon_gen.h
"""
from __future__ import annotations

import itertools
import sys
from fractions import Fraction

import sympy as sp

R = sp.Rational


# ------------------------------------------------------------ helpers
import struct

# FP64 constants that an instruction cannot encode directly (their low 32
# bits are not zero) are collected into one table: on the device the table
# is copied into LDS once per work group and read with broadcast LDS loads,
# instead of being rebuilt in scalar registers at every use.
_KTAB = []
_KIDX = {}


def _encodable(f: float) -> bool:
    return (struct.unpack("<Q", struct.pack("<d", f))[0] & 0xFFFFFFFF) == 0


def lit(x) -> str:
    x = sp.nsimplify(x)
    if x.is_Rational:
        f = float(Fraction(int(x.p), int(x.q)))   # correctly rounded
    else:
        f = float(sp.N(x, 60))
    if f == 0.0:
        return "0.0"
    if _encodable(f):
        return f.hex()
    a = abs(f)
    if a not in _KIDX:
        _KIDX[a] = len(_KTAB)
        _KTAB.append(a)
    return ("-" if f < 0 else "") + f"MR_KT({_KIDX[a]})"


def mono_avg(n, d):
    a, b = R(d) - R(1, 2), R(d) + R(1, 2)
    return (b ** (n + 1) - a ** (n + 1)) / (n + 1)


def mono_mom(n, d):
    return mono_avg(n + 1, d) - d * mono_avg(n, d)


def dot_code(terms, indent="  "):
    """terms: list of (coef (Rational), expr str) -> C expression string."""
    terms = [(c, e) for c, e in terms if c != 0]
    if not terms:
        return "0.0"
    parts = []
    for c, e in terms:
        if c == 1:
            parts.append(f"{e}")
        elif c == -1:
            parts.append(f"-{e}")
        else:
            parts.append(f"{lit(c)} * {e}")
    s = " + ".join(parts)
    return s.replace("+ -", "- ")


# ================================================================== 1D
def maps_1d():
    """q_l coefficient maps over data (um, u0, up, vm, v0, vp)."""
    data = sp.symbols("um u0 up vm v0 vp")
    conds = {2: [(0, -1), (0, 0), (0, 1)],
             3: [(0, -1), (0, 0), (0, 1), (1, 0)],
             4: [(0, -1), (0, 0), (0, 1), (1, -1), (1, 0), (1, 1)]}
    didx = {(0, -1): 0, (0, 0): 1, (0, 1): 2, (1, -1): 3, (1, 0): 4, (1, 1): 5}
    deg = {2: 2, 3: 3, 4: 5}
    out = {}
    for l, cl in conds.items():
        n = deg[l] + 1
        A = sp.Matrix([[mono_avg(p, d) if t == 0 else mono_mom(p, d) for p in range(n)] for t, d in cl])
        b = sp.Matrix([data[didx[c]] for c in cl])
        sol = A.LUsolve(b)
        out[l] = [sp.Poly(sp.expand(s), *data) for s in sol]
    return data, out


def gram_1d(kappa, n):
    G = sp.zeros(n, n)
    for a in range(1, kappa + 1):
        for p in range(a, n):
            for s in range(a, n):
                fp = sp.ff(p, a)
                fs = sp.ff(s, a)
                G[p, s] += fp * fs * mono_avg(p + s - 2 * a, 0)
    return G


def quad_form_code(name, G, idx, var, lines, acc):
    """Emit acc = sum_{p,s in idx} G[p,s] var[p] var[s] with symmetric
    folding: t_p = G_pp v_p + 2 sum_{s>p} G_ps v_s; acc += t_p v_p."""
    first = True
    for a, p in enumerate(idx):
        terms = [(G[p, p], f"{var}[{p}]")]
        for s in idx[a + 1:]:
            terms.append((2 * G[p, s], f"{var}[{s}]"))
        terms = [(c, e) for c, e in terms if c != 0]
        if not terms:
            continue
        lines.append(f"  {{ const double t = {dot_code(terms)};")
        if first:
            lines.append(f"    {acc} = t * {var}[{p}]; }}")
            first = False
        else:
            lines.append(f"    {acc} = fma(t, {var}[{p}], {acc}); }}")
    if first:
        lines.append(f"  {acc} = 0.0;")


def emit_1d(lines):
    data, maps = maps_1d()
    names = ["um", "u0", "up", "vm", "v0", "vp"]
    lines.append("/* ---- 1D: q_2 (3 coefs), q_3 (4), q_4 (6) of eq. (q) ---- */")
    lines.append("MR_DEV inline void mr1_maps(double um, double u0, double up, double vm, double v0, double vp,")
    lines.append("                            double q2[3], double q3[4], double q4[6]) {")
    # parity combos
    lines.append("  const double su = um + up, du = up - um, sv = vm + vp, dv = vp - vm;")
    sym = {"su": None}
    for l, arr in ((2, "q2"), (3, "q3"), (4, "q4")):
        for k, poly in enumerate(maps[l]):
            expr = poly.as_expr()
            # rewrite in terms of (u0, su, du, v0, sv, dv)
            um, u0, up, vm, v0, vp = data
            su, du, sv, dv = sp.symbols("su du sv dv")
            e = sp.expand(expr.subs({um: (su - du) / 2, up: (su + du) / 2, vm: (sv - dv) / 2, vp: (sv + dv) / 2}))
            pe = sp.Poly(e, u0, su, du, v0, sv, dv)
            terms = []
            for sname, s in (("u0", u0), ("su", su), ("du", du), ("v0", v0), ("sv", sv), ("dv", dv)):
                terms.append((pe.coeff_monomial(s), sname))
            lines.append(f"  {arr}[{k}] = {dot_code(terms)};")
    lines.append("}")
    # beta forms
    for kappa, n, nm in ((2, 3, "mr1_beta_k2"), (3, 4, "mr1_beta_k3"), (5, 6, "mr1_beta_k5")):
        G = gram_1d(kappa, n)
        lines.append(f"MR_DEV inline double {nm}(const double c[{n}]) {{")
        lines.append("  double b;")
        quad_form_code(nm, G, list(range(1, n)), "c", lines, "b")
        lines.append("  return b;")
        lines.append("}")
    # evaluation at the 4 GL nodes, parity split
    lines.append("/* values at xi = -1/2, -sqrt(5)/10, sqrt(5)/10, 1/2 of a quintic */")
    lines.append("MR_DEV inline void mr1_eval(const double c[6], double out[4]) {")
    s5 = sp.sqrt(5) / 10
    for nm_, x in (("a", R(1, 2)), ("b", s5)):
        ev = [(sp.nsimplify(x ** k), f"c[{k}]") for k in (0, 2, 4)]
        od = [(sp.nsimplify(x ** k), f"c[{k}]") for k in (1, 3, 5)]
        lines.append(f"  const double e{nm_} = {dot_code(ev)};")
        lines.append(f"  const double o{nm_} = {dot_code(od)};")
    lines.append("  out[0] = ea - oa; out[1] = eb - ob; out[2] = eb + ob; out[3] = ea + oa;")
    lines.append("}")


# ================================================================== 2D
def monos(deg):
    out = []
    for d in range(deg + 1):
        for a in range(d, -1, -1):
            out.append((a, d - a))
    return out


MON = monos(5)   # 21 monomials; P2 = first 6, P3 = first 10


def lab_off(lab):
    return (lab - 1) % 3 - 1, (lab - 1) // 3 - 1


def cond_row(t, lab, a, b):
    dx, dy = lab_off(lab)
    if t == 0:
        return mono_avg(a, dx) * mono_avg(b, dy)
    if t == 1:
        return mono_mom(a, dx) * mono_avg(b, dy)
    return mono_avg(a, dx) * mono_mom(b, dy)


def lsq_map_2d(ncoef, conds):
    """Exact constrained least-squares map: coefficient = M @ data, data are
    the condition values in the order of conds; centre average exact."""
    rows = [[cond_row(t, lab, *MON[p]) for p in range(ncoef)] for t, lab in conds]
    ctr = conds.index((0, 5))
    n = ncoef + 1
    K = sp.zeros(n, n)
    Rhs = sp.zeros(n, len(conds))
    for r, (t, lab) in enumerate(conds):
        if r == ctr:
            for p in range(ncoef):
                K[ncoef, p] = rows[r][p]
                K[p, ncoef] = rows[r][p]
            Rhs[ncoef, r] = 1
            continue
        for p in range(ncoef):
            for s in range(ncoef):
                K[p, s] += rows[r][p] * rows[r][s]
            Rhs[p, r] += rows[r][p]
    sol = K.LUsolve(Rhs)
    return sol[:ncoef, :]


# stencil data symbols: u1..u9, v1..v9, w1..w9 (labels)
U = sp.symbols("u1:10")
V = sp.symbols("v1:10")
W = sp.symbols("w1:10")


def parity_vars():
    """Even/odd combinations of the 3x3 data.  Returns (defs, subs) where
    defs are C definitions and subs maps each raw symbol to an expression in
    the combination symbols."""
    defs = []
    subs = {}
    # averages: a(dx, dy) at label 1 + (dx+1) + 3(dy+1)
    def lab(dx, dy):
        return 1 + (dx + 1) + 3 * (dy + 1)
    combos = {}
    # x-stage for each row dy: e = a(-1)+a(1), o = a(1)-a(-1), c = a(0)
    # y-stage: f_even = f(-1)+f(1), f_odd = f(1)-f(-1), f_mid = f(0)
    # u: classes by (x part, y part)
    syms = {}
    for base, arr in (("u", U),):
        for xp in ("c", "e", "o"):
            for yp in ("m", "s", "d"):
                syms[f"{base}{xp}{yp}"] = sp.Symbol(f"{base}{xp}{yp}")
    # inverse relations: a(dx,dy) in terms of combos
    # x: a(-1) = (e - o)/2, a(1) = (e + o)/2, a(0) = c
    # y: f(-1) = (s - d)/2, f(1) = (s + d)/2, f(0) = m
    def xy_inv(base, dx, dy, xparts=("c", "e", "o")):
        if dy == 0:
            ypart = lambda xp: syms[f"{base}{xp}m"]
        elif dy == -1:
            ypart = lambda xp: (syms[f"{base}{xp}s"] - syms[f"{base}{xp}d"]) / 2
        else:
            ypart = lambda xp: (syms[f"{base}{xp}s"] + syms[f"{base}{xp}d"]) / 2
        if dx == 0:
            return ypart("c")
        if dx == -1:
            return (ypart("e") - ypart("o")) / 2
        return (ypart("e") + ypart("o")) / 2
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            subs[U[lab(dx, dy) - 1]] = xy_inv("u", dx, dy)
    return syms, subs


def emit_2d(lines):
    nco = {2: 6, 3: 10, 4: 21}
    vl = [1, 3, 4, 5, 6, 7, 9]
    wl = [1, 2, 3, 5, 7, 8, 9]
    conds = {2: [(0, l) for l in range(1, 10)],
             3: [(0, l) for l in range(1, 10)] + [(1, 5), (2, 5)],
             4: [(0, l) for l in range(1, 10)] + [(1, l) for l in vl] + [(2, l) for l in wl]}

    def dsym(t, lab):
        return (U, V, W)[t][lab - 1]

    # ---- change of variables to even/odd combinations ----
    # averages
    def lab(dx, dy):
        return 1 + (dx + 1) + 3 * (dy + 1)
    cdefs = []
    cvars = {}
    raw = {}
    def add(name, expr_c, sym_expr):
        cvars[name] = sp.Symbol(name)
        cdefs.append((name, expr_c))
        raw[name] = sym_expr
    # u combos
    for dy in (-1, 0, 1):
        pass
    # explicit: x-stage per row
    def u_(dx, dy):
        return f"u[{lab(dx, dy) - 1}]"
    def v_(dx, dy):
        return f"v[{lab(dx, dy) - 1}]"
    def w_(dx, dy):
        return f"w[{lab(dx, dy) - 1}]"
    # averages: rows (dy) -> e, o, c
    for dy, tag in ((-1, "b"), (0, "m"), (1, "t")):
        add(f"ue{tag}", f"{u_(-1, dy)} + {u_(1, dy)}", U[lab(-1, dy) - 1] + U[lab(1, dy) - 1])
        add(f"uo{tag}", f"{u_(1, dy)} - {u_(-1, dy)}", U[lab(1, dy) - 1] - U[lab(-1, dy) - 1])
    comb = []
    # y-stage
    def ystage(prefix, cen):
        # cen: dict tag->(cexpr, symexpr) for rows b,m,t
        pass
    U5 = U[4]
    final_u = {
        "a00": (f"{u_(0, 0)}", U5),
        "a01": (f"{u_(0, -1)} + {u_(0, 1)}", U[lab(0, -1) - 1] + U[lab(0, 1) - 1]),
        "a02": ("uem", raw["uem"]),
        "a03": ("ueb + uet", raw["ueb"] + raw["uet"]),
        "a10": ("uom", raw["uom"]),
        "a11": ("uob + uot", raw["uob"] + raw["uot"]),
        "a20": (f"{u_(0, 1)} - {u_(0, -1)}", U[lab(0, 1) - 1] - U[lab(0, -1) - 1]),
        "a21": ("uet - ueb", raw["uet"] - raw["ueb"]),
        "a30": ("uot - uob", raw["uot"] - raw["uob"]),
    }
    # classes: a0x -> (0,0), a1x -> (1,0), a2x -> (0,1), a3x -> (1,1)
    # vtilde: available at (+-1, dy) and (0, 0)
    for dy, tag in ((-1, "b"), (0, "m"), (1, "t")):
        add(f"vs{tag}", f"{v_(1, dy)} + {v_(-1, dy)}", V[lab(1, dy) - 1] + V[lab(-1, dy) - 1])
        add(f"vd{tag}", f"{v_(1, dy)} - {v_(-1, dy)}", V[lab(1, dy) - 1] - V[lab(-1, dy) - 1])
    final_v = {
        "b00": ("vdm", raw["vdm"]),                         # (0,0)
        "b01": ("vdb + vdt", raw["vdb"] + raw["vdt"]),      # (0,0)
        "b10": ("vsm", raw["vsm"]),                         # (1,0)
        "b11": ("vsb + vst", raw["vsb"] + raw["vst"]),      # (1,0)
        "b12": (f"{v_(0, 0)}", V[4]),                       # (1,0)
        "b20": ("vdt - vdb", raw["vdt"] - raw["vdb"]),      # (0,1)
        "b30": ("vst - vsb", raw["vst"] - raw["vsb"]),      # (1,1)
    }
    # wtilde: available at (dx, +-1) and (0, 0); mirror of vtilde
    for dx, tag in ((-1, "l"), (0, "m"), (1, "r")):
        add(f"ws{tag}", f"{w_(dx, 1)} + {w_(dx, -1)}", W[lab(dx, 1) - 1] + W[lab(dx, -1) - 1])
        add(f"wd{tag}", f"{w_(dx, 1)} - {w_(dx, -1)}", W[lab(dx, 1) - 1] - W[lab(dx, -1) - 1])
    final_w = {
        "c00": ("wdm", raw["wdm"]),                         # (0,0)
        "c01": ("wdl + wdr", raw["wdl"] + raw["wdr"]),      # (0,0)
        "c20": ("wsm", raw["wsm"]),                         # (0,1)
        "c21": ("wsl + wsr", raw["wsl"] + raw["wsr"]),      # (0,1)
        "c22": (f"{w_(0, 0)}", W[4]),                       # (0,1)
        "c10": ("wdr - wdl", raw["wdr"] - raw["wdl"]),      # (1,0)
        "c30": ("wsr - wsl", raw["wsr"] - raw["wsl"]),      # (1,1)
    }
    finals = {}
    finals.update(final_u)
    finals.update(final_v)
    finals.update(final_w)
    # express the raw data in terms of the final combination variables:
    # solve the linear system raw -> finals (exact)
    fin_names = list(finals.keys())
    fin_syms = sp.symbols(" ".join(fin_names))
    used_raw = list(U) + [V[l - 1] for l in vl] + [W[l - 1] for l in wl]
    eqs = [sp.Eq(fs, finals[n][1]) for n, fs in zip(fin_names, fin_syms)]
    sol = sp.solve(eqs, used_raw, dict=True)[0]

    lines.append("/* ---- 2D: q_2 (6 coefs), q_3 (10), q_4 (21) of eqs. (2D-q2)-(2D-q4),")
    lines.append("   centre average exact, other conditions in the least-squares sense.")
    lines.append("   Monomial order: degree by degree, xi power descending:")
    lines.append("   " + ", ".join(f"x^{a}y^{b}" for a, b in MON) + " */")
    lines.append("MR_DEV inline void mr2_maps(const double u[9], const double v[9], const double w[9],")
    lines.append("                            double q2[6], double q3[10], double q4[21]) {")
    for name, cexpr in cdefs:
        lines.append(f"  const double {name} = {cexpr};")
    for n in fin_names:
        cexpr = finals[n][0]
        lines.append(f"  const double {n} = {cexpr};")
    total_terms = 0
    for l, arr in ((2, "q2"), (3, "q3"), (4, "q4")):
        M = lsq_map_2d(nco[l], conds[l])
        datas = [dsym(t, lb) for t, lb in conds[l]]
        for p in range(nco[l]):
            expr = sum(M[p, k] * datas[k] for k in range(len(datas)))
            e = sp.expand(expr.subs(sol))
            terms = [(e.coeff(fs), n) for n, fs in zip(fin_names, fin_syms)]
            # sanity: nothing left over
            rest = sp.expand(e - sum(c * fs for c, (nn, fs) in zip([t[0] for t in terms], zip(fin_names, fin_syms))))
            assert rest == 0, rest
            total_terms += sum(1 for c, _ in terms if c != 0)
            lines.append(f"  {arr}[{p}] = {dot_code(terms)};")
    lines.append(f"  /* {total_terms} non-zero map entries after the parity split */")
    lines.append("}")

    # ---- beta quadratic forms, blocks by parity class ----
    def gram2(kappa, n):
        G = sp.zeros(n, n)
        for ax in range(0, kappa + 1):
            for ay in range(0, kappa + 1 - ax):
                if ax + ay == 0:
                    continue
                for p in range(n):
                    a1, b1 = MON[p]
                    if a1 < ax or b1 < ay:
                        continue
                    for s in range(n):
                        a2, b2 = MON[s]
                        if a2 < ax or b2 < ay:
                            continue
                        G[p, s] += (sp.ff(a1, ax) * sp.ff(a2, ax) * sp.ff(b1, ay) * sp.ff(b2, ay)
                                    * mono_avg(a1 + a2 - 2 * ax, 0) * mono_avg(b1 + b2 - 2 * ay, 0))
        return G
    for kappa, n, nm in ((2, 6, "mr2_beta_k2"), (3, 10, "mr2_beta_k3"), (5, 21, "mr2_beta_k5")):
        G = gram2(kappa, n)
        lines.append(f"MR_DEV inline double {nm}(const double c[{n}]) {{")
        lines.append("  double b = 0.0, part;")
        for cls in ((0, 0), (1, 0), (0, 1), (1, 1)):
            idx = [p for p in range(1, n) if (MON[p][0] % 2, MON[p][1] % 2) == cls]
            # check block structure
            for p in idx:
                for s in range(1, n):
                    if s not in idx:
                        assert G[p, s] == 0
            if not idx:
                continue
            quad_form_code(nm, G, idx, "c", lines, "part")
            lines.append("  b += part;")
        lines.append("  return b;")
        lines.append("}")

    # ---- evaluation at the 4x4 Gauss-Lobatto grid ----
    s5 = sp.sqrt(5) / 10
    absn = [R(1, 2), s5]      # |node| for k = 0/3 and 1/2
    lines.append("/* values of a degree-5 polynomial at (xi_k, eta_l), out[k + 4 l],")
    lines.append("   xi, eta in {-1/2, -sqrt(5)/10, sqrt(5)/10, 1/2} */")
    lines.append("MR_DEV inline void mr2_eval(const double c[21], double out[16]) {")
    # class values at |xi| = A/B, |eta| = A/B
    for ix, X in enumerate(absn):
        for iy, Y in enumerate(absn):
            for cls in ((0, 0), (1, 0), (0, 1), (1, 1)):
                terms = []
                for p, (a, b) in enumerate(MON):
                    if (a % 2, b % 2) == cls:
                        terms.append((sp.nsimplify(X ** a * Y ** b), f"c[{p}]"))
                lines.append(f"  const double P{cls[0]}{cls[1]}_{ix}{iy} = {dot_code(terms)};")
    # node index k: 0 -> -A, 1 -> -B, 2 -> +B, 3 -> +A  (A = 1/2 -> ix 0, B -> ix 1)
    node = {0: (0, -1), 1: (1, -1), 2: (1, 1), 3: (0, 1)}
    for l in range(4):
        for k in range(4):
            ix, sx = node[k]
            iy, sy = node[l]
            t = f"P00_{ix}{iy}"
            t += (" + " if sx > 0 else " - ") + f"P10_{ix}{iy}"
            t += (" + " if sy > 0 else " - ") + f"P01_{ix}{iy}"
            t += (" + " if sx * sy > 0 else " - ") + f"P11_{ix}{iy}"
            lines.append(f"  out[{k + 4 * l}] = {t};")
    lines.append("}")


def emit_mod(lines):
    """Step 2.2, eqs. (p0)/(vi): first moment of the quartic p_0."""
    c = sp.symbols("p0:5")
    conds = [(0, -1), (0, 0), (0, 1), (1, -1), (1, 1)]
    A = sp.Matrix([[mono_avg(p, d) if t == 0 else mono_mom(p, d) for p in range(5)] for t, d in conds])
    um, u0, up, vm, vp = sp.symbols("um u0 up vm vp")
    sol = A.LUsolve(sp.Matrix([um, u0, up, vm, vp]))
    vnew = sp.expand(sum(sol[p] * mono_mom(p, 0) for p in range(5)))
    cu = vnew.coeff(up)
    cv = vnew.coeff(vm)
    assert vnew.coeff(um) == -cu and vnew.coeff(vp) == cv and vnew.coeff(u0) == 0
    lines.append(f"/* modified first moment: {cu} (u_+ - u_-) + ({cv}) (v_- + v_+) */")
    lines.append("MR_DEV inline double mr_modified_moment(double um, double up, double vm, double vp) {")
    lines.append(f"  return {lit(cu)} * (up - um) + {lit(cv)} * (vm + vp);")
    lines.append("}")


def main():
    body = []
    emit_mod(body)
    emit_1d(body)
    emit_2d(body)
    lines = ["/* Generated by gen_recon.py -- do not edit. */",
             "#pragma once",
             "#ifndef MR_DEV",
             "#define MR_DEV __host__ __device__ __attribute__((always_inline))",
             "#endif",
             f"#define MR_NKT {len(_KTAB)}",
             "/* constants the instructions cannot encode; MR_KT(i) reads entry i",
             "   (the including file defines MR_KT and the table storage) */",
             "#define MR_KT_VALUES \\"]
    for k in range(0, len(_KTAB), 4):
        lines.append("  " + ", ".join(v.hex() for v in _KTAB[k:k + 4]) + ", \\")
    lines.append("  0.0")
    lines.append("MR_KT_DECLARE")
    lines.append("")
    lines.extend(body)
    sys.stdout.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
