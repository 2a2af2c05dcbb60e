"""Index-data patterns for the stage-pattern front end (eq. 3: one algebraic
pattern evaluated at many discretization points, differing only in the data
it reads).

A PatternModel writes a stage's rows and objective as a few templates, each
instantiated over a table: an instance names the stage variables bound to the
template's variable slots, the previous-stage states bound to its previous
slots, numeric data, setpoint entries and (for rows) the state whose equation
it is.  The templates are differentiated once; the generated kernels give
every instance of a pattern the same code (no divergence within a pattern),
reading their bindings from tables compiled into the code object.  Rows own
their Jacobian entries; the Hessian, gradient and objective contributions of
the instances go to a per-stage scratch array and a second generated kernel
sums them per Hessian slot, gradient entry and stage in a fixed order.

Pattern kinds follow eq. (3): state rows (the differential patterns, one per
state), algebraic equality rows, inequality rows d <= 0, and objective terms.
Previous states enter state rows only, linearly with constant coefficients;
rows read variables, data and dt; objective templates may also read setpoint
entries and the stage's trajectory value.  The cold-start guess is the
measured state and the last control, and for algebraic variables a guess
pattern over measured states, last controls and data (0 where none is given).
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

from .simd import (GeneratedModel, _Emitter, _header_text, _tag, add, diff, is_const, lift, mul, neg,
                   sym, symbols)


def _kinds(e):
    return {s.args[0] for s in symbols(e)}


@dataclass
class Pattern:
    kind: str            # "row" (state rows), "alg" (algebraic rows), "ineq" or "obj"
    expr: object
    nv: int
    nprev: int
    ndata: int
    nsp: int
    instances: list      # dicts: vars, prevs, data, sps, target, pus
    npu: int = 0         # objective: slots of the previous stage's controls


@dataclass
class GuessPattern:
    expr: object
    nx0: int
    nup: int
    ndata: int
    instances: list      # dicts: target (algebraic variable), x0s, ups, data


@dataclass
class PatternModel:
    """Stage layout [states | controls | algebraic variables]; every state's
    row comes from exactly one instance of a state-row pattern."""
    name: str
    n_setpoint: int = 0
    uses_traj: bool = False
    lb: list = field(default_factory=list)
    ub: list = field(default_factory=list)
    nx: int = 0
    nu: int = 0
    na: int = 0
    patterns: list = field(default_factory=list)
    guesses: list = field(default_factory=list)

    def states(self, count, lb=-math.inf, ub=math.inf):
        if self.nu or self.na:
            raise ValueError("declare the states before the controls and algebraic variables")
        first = self.nx
        self.nx += count
        self.lb += [float(lb)] * count
        self.ub += [float(ub)] * count
        return list(range(first, first + count))

    def controls(self, count, lb=-math.inf, ub=math.inf):
        if self.na:
            raise ValueError("declare the controls before the algebraic variables")
        first = self.nx + self.nu
        self.nu += count
        self.lb += [float(lb)] * count
        self.ub += [float(ub)] * count
        return list(range(first, first + count))

    def algebraic(self, count, lb=-math.inf, ub=math.inf):
        first = self.ns
        self.na += count
        self.lb += [float(lb)] * count
        self.ub += [float(ub)] * count
        return list(range(first, first + count))

    @property
    def ns(self):
        return self.nx + self.nu + self.na

    @property
    def dt(self):
        return sym("dt")

    def traj(self):
        self.uses_traj = True
        return sym("tr")

    def row_pattern(self, template, instances, nv, nprev=0, ndata=0):
        """template(v, p, d) -> residual; v: nv variable slots, p: nprev
        previous-state slots, d: ndata numeric data.  instances: dicts with
        target (state index), vars (nv stage-variable indices, distinct), prevs
        (nprev state indices), data (ndata floats)."""
        v = [sym("sv", j) for j in range(nv)]
        p = [sym("sprev", j) for j in range(nprev)]
        d = [sym("sd", j) for j in range(ndata)]
        self.patterns.append(Pattern("row", lift(template(v, p, d)), nv, nprev, ndata, 0, list(instances)))

    def algebraic_row_pattern(self, template, instances, nv, ndata=0):
        """template(v, d) -> residual of an equality row within the stage (no
        previous states); one row per instance, numbered in declaration order.
        instances: dicts with vars and data."""
        v = [sym("sv", j) for j in range(nv)]
        d = [sym("sd", j) for j in range(ndata)]
        self.patterns.append(Pattern("alg", lift(template(v, d)), nv, 0, ndata, 0, list(instances)))

    def inequality_pattern(self, template, instances, nv, ndata=0):
        """template(v, d) -> d_row, the row d_row <= 0; one per instance."""
        v = [sym("sv", j) for j in range(nv)]
        d = [sym("sd", j) for j in range(ndata)]
        self.patterns.append(Pattern("ineq", lift(template(v, d)), nv, 0, ndata, 0, list(instances)))

    def guess_pattern(self, template, instances, nx0=0, nup=0, ndata=0):
        """template(x, u, d) -> cold-start value of an algebraic variable from
        measured-state slots x, last-control slots u and data d.  instances:
        dicts with target (algebraic variable), x0s (state indices), ups
        (control numbers, 0-based), data."""
        x = [sym("sx0", j) for j in range(nx0)]
        u = [sym("sup", j) for j in range(nup)]
        d = [sym("sd", j) for j in range(ndata)]
        self.guesses.append(GuessPattern(lift(template(x, u, d)), nx0, nup, ndata, list(instances)))

    def generate(self):
        return generate(self)

    def objective_pattern(self, template, instances, nv, ndata=0, nsp=0, npu=0):
        """template(v, d, s) -> stage term, or template(v, d, s, pu) with npu
        > 0; s: nsp setpoint slots; pu: slots of the previous stage's controls
        (the last applied control at the first stage), as move penalties use.
        instances: dicts with vars, data, sps (setpoint indices), pus (control
        numbers, 0-based)."""
        v = [sym("sv", j) for j in range(nv)]
        d = [sym("sd", j) for j in range(ndata)]
        s = [sym("ssp", j) for j in range(nsp)]
        args = (v, d, s) if npu == 0 else (v, d, s, [sym("spu", j) for j in range(npu)])
        self.patterns.append(Pattern("obj", lift(template(*args)), nv, 0, ndata, nsp, list(instances), npu))


# ---- derivation --------------------------------------------------------------------
@dataclass
class PatternDerived:
    pat: Pattern
    dv: list             # d expr / d sv_j
    pcoef: list          # constant d expr / d sprev_j (rows)
    pairs: list          # (j, l) slot pairs with a nonzero second derivative
    d2: list             # their expressions (times the row multiplier for rows)
    dpu: list = None     # objective: d expr / d spu_b
    xpairs: list = None  # (variable slot j, previous-control slot b) with a nonzero second derivative
    xd2: list = None
    ppairs: list = None  # (b, b2), b >= b2: previous-control pairs (the previous stage's Hessian)
    pd2: list = None


_ALLOWED = {"row": {"sv", "sprev", "sd", "dt", "tr"}, "alg": {"sv", "sd", "dt", "tr"}, "ineq": {"sv", "sd", "dt", "tr"},
            "obj": {"sv", "sd", "ssp", "tr", "dt", "spu"}}


def _derive_pattern(pat: Pattern):
    allowed = _ALLOWED[pat.kind]
    bad = _kinds(pat.expr) - allowed
    if bad:
        raise ValueError(f"a {pat.kind} pattern uses {sorted(bad)}")
    memo = {}
    V = [sym("sv", j) for j in range(pat.nv)]
    dv = [diff(pat.expr, v, memo.setdefault(v, {})) for v in V]
    pcoef = []
    for j in range(pat.nprev):
        c = diff(pat.expr, sym("sprev", j))
        if not is_const(c) or is_const(c, 0.0):
            raise ValueError("previous-state slots must enter linearly with nonzero constant coefficients")
        pcoef.append(c.args[0])
    pairs, d2 = [], []
    for j in range(pat.nv):
        for l in range(j + 1):
            e = diff(dv[j], V[l])
            if not is_const(e, 0.0):
                pairs.append((j, l))
                d2.append(e)
    PU = [sym("spu", b) for b in range(pat.npu)]
    dpu = [diff(pat.expr, u, memo.setdefault(u, {})) for u in PU]
    xpairs, xd2, ppairs, pd2 = [], [], [], []
    for j in range(pat.nv):
        for b in range(pat.npu):
            e = diff(dv[j], PU[b])
            if not is_const(e, 0.0):
                xpairs.append((j, b))
                xd2.append(e)
    for b in range(pat.npu):
        for b2 in range(b + 1):
            e = diff(dpu[b], PU[b2])
            if not is_const(e, 0.0):
                ppairs.append((b, b2))
                pd2.append(e)
    return PatternDerived(pat, dv, pcoef, pairs, d2, dpu, xpairs, xd2, ppairs, pd2)


def _structure(m: PatternModel, ders):
    """Per-stage patterns, per-instance Jacobian positions, the Hessian slots
    and the scratch layout with the reduction lists."""
    ns, nx = m.ns, m.nx
    rows = [None] * nx
    for pi, dd in enumerate(ders):
        if dd.pat.kind != "row":
            continue
        for ii, inst in enumerate(dd.pat.instances):
            t = int(inst["target"])
            if not 0 <= t < nx or rows[t] is not None:
                raise ValueError(f"state {t}: no or several row instances")
            vs = [int(v) for v in inst["vars"]]
            if len(vs) != dd.pat.nv or len(set(vs)) != len(vs) or not all(0 <= v < ns for v in vs):
                raise ValueError(f"row of state {t}: variable slots must be distinct stage variables")
            if t not in vs:
                raise ValueError(f"row of state {t} does not hold its own state")
            ps = [int(q) for q in inst.get("prevs", [])]
            if len(ps) != dd.pat.nprev or len(set(ps)) != len(ps) or not all(0 <= q < nx for q in ps):
                raise ValueError(f"row of state {t}: previous slots must be distinct states")
            if len(inst.get("data", [])) != dd.pat.ndata:
                raise ValueError(f"row of state {t}: wrong number of data values")
            rows[t] = (pi, ii)
    if any(r is None for r in rows):
        raise ValueError(f"states without a row: {[t for t, r in enumerate(rows) if r is None][:8]} ...")
    # algebraic and inequality rows, numbered in declaration order
    arow, drow = {}, {}
    for pi, dd in enumerate(ders):
        if dd.pat.kind not in ("alg", "ineq"):
            continue
        for ii, inst in enumerate(dd.pat.instances):
            vs = [int(v) for v in inst["vars"]]
            if len(vs) != dd.pat.nv or len(set(vs)) != len(vs) or not all(0 <= v < ns for v in vs):
                raise ValueError(f"{dd.pat.kind} row: variable slots must be distinct stage variables")
            if len(inst.get("data", [])) != dd.pat.ndata:
                raise ValueError(f"{dd.pat.kind} row: wrong number of data values")
            if dd.pat.kind == "alg":
                arow[(pi, ii)] = nx + len(arow)
            else:
                drow[(pi, ii)] = len(drow)
    rows = rows + [None] * len(arow)
    for key, r in arow.items():
        rows[r] = key
    # per-row columns (own sorted; previous sorted) and slot positions
    row_ptr, row_cols, prev_ptr, prev_cols, prev_coef = [0], [], [0], [], []
    jpos, ppos = {}, {}
    for t in range(len(rows)):
        pi, ii = rows[t]
        dd = ders[pi]
        inst = dd.pat.instances[ii]
        own = sorted(int(v) for v in inst["vars"])
        row_cols += own
        row_ptr.append(len(row_cols))
        pv = [int(q) for q in inst.get("prevs", [])]
        order = sorted(range(len(pv)), key=lambda j: pv[j])
        prev_cols += [pv[j] for j in order]
        prev_coef += [dd.pcoef[j] for j in order]
        prev_ptr.append(len(prev_cols))
        jpos[(pi, ii)] = [own.index(int(v)) for v in inst["vars"]]
        ppos[(pi, ii)] = [order.index(j) for j in range(len(pv))]
    ineq_ptr, ineq_cols = [0], []
    for (pi, ii), d in sorted(drow.items(), key=lambda kv: kv[1]):
        own = sorted(int(v) for v in ders[pi].pat.instances[ii]["vars"])
        ineq_cols += own
        ineq_ptr.append(len(ineq_cols))
        jpos[(pi, ii)] = [own.index(int(v)) for v in ders[pi].pat.instances[ii]["vars"]]
    # Hessian slots: lower pairs of stage variables over all instances (the
    # previous-control pairs of objective terms land in the previous stage's
    # own slots), and pairs (stage variable, previous stage's control)
    wkeys, xkeys = {}, {}
    for pi, dd in enumerate(ders):
        for inst in dd.pat.instances:
            vs = [int(v) for v in inst["vars"]]
            pus = [int(b) for b in inst.get("pus", [])]
            for (j, l) in dd.pairs:
                a, b = max(vs[j], vs[l]), min(vs[j], vs[l])
                wkeys.setdefault((a, b), None)
            for (b, b2) in (dd.ppairs or []):
                a, c = nx + max(pus[b], pus[b2]), nx + min(pus[b], pus[b2])
                wkeys.setdefault((a, c), None)
            for (j, b) in (dd.xpairs or []):
                xkeys.setdefault((vs[j], pus[b]), None)
    wlist = sorted(wkeys)
    widx = {k: i for i, k in enumerate(wlist)}
    xlist = sorted(xkeys)
    xidx = {k: i for i, k in enumerate(xlist)}
    # scratch of a stage: per pattern, entry c of instance i at base + c n + i
    # (n instances; consecutive lanes write consecutive doubles).  Entries: the
    # Hessian contributions, then (objective) the gradient contributions and
    # the value.  The objective values are spread over the stage's NS
    # objective-term slots (value of the f-th instance overall -> slot f % NS).
    # Objective instances with previous-control slots add, after their own
    # entries, the cross pairs, the previous-control pairs and the gradient
    # in the previous controls; the last two are summed by the previous
    # stage's lanes (lists wn_lists, gn_lists over the next stage's scratch).
    coo_base, ncoo = [], 0
    w_lists = [[] for _ in wlist]
    wn_lists = [[] for _ in wlist]
    x_lists = [[] for _ in xlist]
    g_lists = [[] for _ in range(ns)]
    gn_lists = [[] for _ in range(ns)]
    f_lists = [[] for _ in range(ns)]
    nf = 0
    offs = []
    for pi, dd in enumerate(ders):
        n = len(dd.pat.instances)
        npr, nxp, npp = len(dd.pairs), len(dd.xpairs or []), len(dd.ppairs or [])
        if dd.pat.kind == "obj":
            o_x = npr + dd.pat.nv + 1          # cross pairs
            o_p = o_x + nxp                    # previous-control pairs
            o_g = o_p + npp                    # gradient in the previous controls
            per = o_g + dd.pat.npu
        else:
            o_x = o_p = o_g = per = npr
        offs.append((o_x, o_p, o_g))
        coo_base.append(ncoo)
        for ii, inst in enumerate(dd.pat.instances):
            vs = [int(v) for v in inst["vars"]]
            pus = [int(b) for b in inst.get("pus", [])]
            for c, (j, l) in enumerate(dd.pairs):
                w_lists[widx[(max(vs[j], vs[l]), min(vs[j], vs[l]))]].append(ncoo + c * n + ii)
            if dd.pat.kind == "obj":
                for j in range(dd.pat.nv):
                    g_lists[vs[j]].append(ncoo + (npr + j) * n + ii)
                f_lists[nf % ns].append(ncoo + (npr + dd.pat.nv) * n + ii)
                nf += 1
                for c, (j, b) in enumerate(dd.xpairs or []):
                    x_lists[xidx[(vs[j], pus[b])]].append(ncoo + (o_x + c) * n + ii)
                for c, (b, b2) in enumerate(dd.ppairs or []):
                    key = (nx + max(pus[b], pus[b2]), nx + min(pus[b], pus[b2]))
                    wn_lists[widx[key]].append(ncoo + (o_p + c) * n + ii)
                for b in range(dd.pat.npu):
                    gn_lists[nx + pus[b]].append(ncoo + (o_g + b) * n + ii)
        ncoo += per * n
    return dict(rows=rows, row_ptr=row_ptr, row_cols=row_cols, prev_ptr=prev_ptr, prev_cols=prev_cols,
                prev_coef=prev_coef, jpos=jpos, ppos=ppos, wlist=wlist, coo_base=coo_base, ncoo=ncoo,
                w_lists=w_lists, g_lists=g_lists, f_lists=f_lists, arow=arow, drow=drow, n_alg=len(arow),
                xlist=xlist, x_lists=x_lists, wn_lists=wn_lists, gn_lists=gn_lists, offs=offs,
                nd=len(drow), ineq_ptr=ineq_ptr, ineq_cols=ineq_cols)


# ---- C emission ---------------------------------------------------------------------------
def _ints(name, vals):
    vals = [int(v) for v in vals] or [0]
    body = ",".join(str(int(v)) for v in vals)
    return f"__device__ const int {name}[{len(vals)}] = {{{body}}};"


def _dbls(name, vals):
    vals = list(vals) or [0.0]
    body = ",".join(repr(float(v)) for v in vals)
    return f"__device__ const double {name}[{len(vals)}] = {{{body}}};"


def _csr(name, lists):
    ptr = [0]
    idx = []
    for l in lists:
        idx += l
        ptr.append(len(idx))
    return _ints(name + "_PTR", ptr) + "\n" + _ints(name + "_IDX", idx)


def _source(m: PatternModel, ders, st, tag: int) -> str:
    nx, nu, ns = m.nx, m.nu, m.ns
    nw, nwx = len(st["wlist"]), len(st["xlist"])
    nlanes = sum(len(d.pat.instances) for d in ders)
    out = []
    w = out.append
    w(f"// Kernels of the pattern model '{m.name}', written by the stage-pattern front end.")
    w("#include \"kernels.h\"")
    w("using namespace nmpc;")
    w("namespace {")
    w(f"constexpr int NS = {ns}, NX = {nx}, NU = {nu}, RPS = {nx + st['n_alg']}, ND = {st['nd']}, NW = {nw}, "
      f"NWX = {nwx}, NCOO = {max(st['ncoo'], 1)}, NLANES = {nlanes}, NSP = {m.n_setpoint};")
    w("// (a model with no Hessian, gradient or objective contributions still has one scratch double")
    w("// per stage, so the summing kernel runs and writes the zeros)")
    w(f"constexpr unsigned long long TAG = {tag}ULL;")
    w("// Hessian slots of stage k: its own NW, then (k > 0) NWX with the previous stage's controls")
    w("__device__ inline int64_t woff(int k) { return k == 0 ? 0 : NW + (int64_t)(k - 1) * (NW + NWX); }")
    w("// binding tables of the instances (instance-major), compiled into the code object")
    for pi, dd in enumerate(ders):
        insts = dd.pat.instances
        w(_ints(f"P{pi}_V", [v for inst in insts for v in inst["vars"]]))
        if dd.pat.nprev:
            w(_ints(f"P{pi}_PV", [q for inst in insts for q in inst["prevs"]]))
            w(_ints(f"P{pi}_PP", [p for ii in range(len(insts)) for p in st["ppos"][(pi, ii)]]))
        if dd.pat.ndata:
            w(_dbls(f"P{pi}_D", [x for inst in insts for x in inst["data"]]))
        if dd.pat.npu:
            w(_ints(f"P{pi}_PU", [b for inst in insts for b in inst["pus"]]))
        if dd.pat.nsp:
            w(_ints(f"P{pi}_SP", [q for inst in insts for q in inst["sps"]]))
            for slot in range(dd.pat.nsp):
                inv = [[] for _ in range(m.n_setpoint)]
                for ii, inst in enumerate(insts):
                    inv[int(inst["sps"][slot])].append(ii)
                w(_csr(f"P{pi}_S{slot}", inv))
        if dd.pat.kind != "obj":   # the row of each instance (stage-local) and its Jacobian slots
            rowno = {"row": lambda ii: insts[ii]["target"], "alg": lambda ii: st["arow"][(pi, ii)],
                     "ineq": lambda ii: st["drow"][(pi, ii)]}[dd.pat.kind]
            w(_ints(f"P{pi}_T", [rowno(ii) for ii in range(len(insts))]))
            w(_ints(f"P{pi}_JP", [p for ii in range(len(insts)) for p in st["jpos"][(pi, ii)]]))
    for gi, gp in enumerate(m.guesses):
        insts = gp.instances
        if gp.nx0:
            w(_ints(f"G{gi}_X", [q for inst in insts for q in inst["x0s"]]))
        if gp.nup:
            w(_ints(f"G{gi}_U", [q for inst in insts for q in inst["ups"]]))
        if gp.ndata:
            w(_dbls(f"G{gi}_D", [x for inst in insts for x in inst["data"]]))
    # guess of each algebraic variable: (guess pattern, instance), or -1
    gsel = [(-1, 0)] * m.na
    for gi, gp in enumerate(m.guesses):
        for ii, inst in enumerate(gp.instances):
            gsel[int(inst["target"]) - nx - nu] = (gi, ii)
    w(_ints("GA_P", [a for a, _ in gsel]))
    w(_ints("GA_I", [b for _, b in gsel]))
    w("// summation lists of a stage's scratch: Hessian slots, gradient entries, objective-term slots;")
    w("// cross slots; and the next stage's entries that belong to this stage's controls")
    w(_csr("RW", st["w_lists"]))
    w(_csr("RG", st["g_lists"]))
    w(_csr("RF", st["f_lists"]))
    w(_csr("RX", st["x_lists"]))
    w(_csr("RWN", st["wn_lists"]))
    w(_csr("RGN", st["gn_lists"]))
    # x0 contraction: the state rows holding each previous state, with coefficients
    xl = [[] for _ in range(nx)]
    for t in range(nx):
        for q in range(st["prev_ptr"][t], st["prev_ptr"][t + 1]):
            xl[st["prev_cols"][q]].append((t, st["prev_coef"][q]))
    w(_ints("XR_PTR", np.concatenate([[0], np.cumsum([len(l) for l in xl])])))
    w(_ints("XR_ROW", [r for l in xl for r, _ in l]))
    w(_dbls("XR_COEF", [c for l in xl for _, c in l]))
    w("}  // namespace")
    w("")
    w("// descriptor layout these kernels were built against (checked at load)")
    w("extern \"C\" __device__ unsigned int nmpc_stage_abi = kStageAbi;")
    w("")
    # evaluation: one lane per (stage, instance), instances fastest, grid-stride
    w("// One lane per (stage, instance), instances fastest: the lanes of a wavefront")
    w("// run one pattern on neighbouring instances of one stage.")
    w("extern \"C\" __global__ void __launch_bounds__(kBlock)")
    w("nmpc_stage_eval(const InstPtrs* __restrict__ Ia, Space sp, int src, int pred, int full) {")
    w("    int lb;")
    w("    const int inst = block_inst(sp, lb);")
    w("    const InstPtrs& I = Ia[inst];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG || !ctl_active(I.ctl, pred)) return;")
    w("    const int lanes = (sp.bfirst[inst + 1] - sp.bfirst[inst]) * kBlock;")
    w("    const double* __restrict__ y = src == kSrcIter ? I.y : I.yt;")
    w("    const double* __restrict__ om = src == kSrcUser ? I.dom : I.om;")
    w("    const double* SP = I.setp;")
    w("    const double DT = I.gm.dt;")
    w("    const int mc = I.mc;")
    w("    (void)SP; (void)DT; (void)om; (void)mc;")
    w("    for (int t = lb * kBlock + threadIdx.x; t < I.H * NLANES; t += lanes) {")
    w("        const int k = t / NLANES, j = t - k * NLANES;")
    w("        const double* V = y + (int64_t)k * NS;")
    w("        const double TR = I.ntr > 0 ? I.zF[k] : 0.0;")
    w("        double* Sk = I.gm.scratch + (int64_t)k * NCOO;")
    w("        (void)V; (void)TR; (void)Sk;")
    start = 0
    for pi, dd in enumerate(ders):
        pat = dd.pat
        n = len(pat.instances)
        base = st["coo_base"][pi]
        w(f"        {'if' if pi == 0 else 'else if'} (j < {start + n}) {{")
        w(f"            const int i = j - {start};")
        names = {"sv": f"V[P{pi}_V[i * {pat.nv} + {{j}}]]", "dt": "DT", "tr": "TR"}
        if pat.ndata:
            names["sd"] = f"P{pi}_D[i * {pat.ndata} + {{j}}]"
        if pat.nsp:
            names["ssp"] = f"SP[P{pi}_SP[i * {pat.nsp} + {{j}}]]"
        if pat.nprev:
            names["sprev"] = (f"(k > 0 ? y[(int64_t)(k - 1) * NS + P{pi}_PV[i * {pat.nprev} + {{j}}]] "
                              f": I.x0[P{pi}_PV[i * {pat.nprev} + {{j}}]])")
        if pat.npu:
            names["spu"] = (f"(k > 0 ? y[(int64_t)(k - 1) * NS + NX + P{pi}_PU[i * {pat.npu} + {{j}}]] "
                            f": I.uprev[P{pi}_PU[i * {pat.npu} + {{j}}]])")
        em = _Emitter(None, names, indent=3)
        if pat.kind == "ineq":
            em.line(f"const int r = k * ND + P{pi}_T[i];")
            em.line(f"I.d[r] = {em.val(pat.expr)};")
            em.line("if (full) {")
            em.indent += 1
            em.push()
            em.line("double* jr = I.jv + I.jptr[mc + r];")
            for s_, e in enumerate(dd.dv):
                em.line(f"jr[P{pi}_JP[i * {pat.nv} + {s_}]] = {em.val(e)};")
            if dd.pairs:
                em.line("const double lam = om[2 * mc + r];")
                for c, e in enumerate(dd.d2):
                    em.line(f"Sk[{base + c * n} + i] = lam * {em.val(e)};")
            em.pop()
            em.indent -= 1
            em.line("}")
        elif pat.kind in ("row", "alg"):
            em.line(f"const int r = k * RPS + P{pi}_T[i];")
            em.line(f"I.c[r] = {em.val(pat.expr)};")
            em.line("if (full) {")
            em.indent += 1
            em.push()
            if pat.nprev:
                em.line(f"double* jr = I.jv + I.jptr[r] + (k > 0 ? {pat.nprev} : 0);")
                em.line("if (k > 0) {")
                for q, c in enumerate(dd.pcoef):
                    em.line(f"    I.jv[I.jptr[r] + P{pi}_PP[i * {pat.nprev} + {q}]] = {c!r};")
                em.line("}")
            else:
                em.line("double* jr = I.jv + I.jptr[r];")
            for s_, e in enumerate(dd.dv):
                em.line(f"jr[P{pi}_JP[i * {pat.nv} + {s_}]] = {em.val(e)};")
            if dd.pairs:
                em.line("const double lam = om[r] - om[mc + r];")
                for c, e in enumerate(dd.d2):
                    em.line(f"Sk[{base + c * n} + i] = lam * {em.val(e)};")
            em.pop()
            em.indent -= 1
            em.line("}")
        else:
            np_ = len(dd.pairs)
            o_x, o_p, o_g = st["offs"][pi]
            em.line(f"Sk[{base + (np_ + pat.nv) * n} + i] = {em.val(pat.expr)};")
            em.line("if (full) {")
            em.indent += 1
            em.push()
            for c, e in enumerate(dd.d2):
                em.line(f"Sk[{base + c * n} + i] = {em.val(e)};")
            for s_, e in enumerate(dd.dv):
                em.line(f"Sk[{base + (np_ + s_) * n} + i] = {em.val(e)};")
            for c, e in enumerate(dd.xd2 or []):
                em.line(f"Sk[{base + (o_x + c) * n} + i] = {em.val(e)};")
            for c, e in enumerate(dd.pd2 or []):
                em.line(f"Sk[{base + (o_p + c) * n} + i] = {em.val(e)};")
            for b_, e in enumerate(dd.dpu or []):
                em.line(f"Sk[{base + (o_g + b_) * n} + i] = {em.val(e)};")
            em.pop()
            em.indent -= 1
            em.line("}")
        out.extend(em.lines)
        w("        }")
        start += n
    w("    }")
    w("}")
    w("")
    # reduction: Hessian slots, gradient entries and objective-term slots, in list order
    w("// Sums of the scratch, one lane per (stage, Hessian slot or variable), in the")
    w("// fixed order of the lists: Hessian values, gradient and objective terms.")
    w("extern \"C\" __global__ void __launch_bounds__(kBlock)")
    w("nmpc_stage_reduce(const InstPtrs* __restrict__ Ia, Space sp, int pred, int full) {")
    w("    int lb;")
    w("    const int inst = block_inst(sp, lb);")
    w("    const InstPtrs& I = Ia[inst];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG || !ctl_active(I.ctl, pred)) return;")
    w("    const int lanes = (sp.bfirst[inst + 1] - sp.bfirst[inst]) * kBlock;")
    w("    for (int t = lb * kBlock + threadIdx.x; t < I.H * (NW + NWX + NS); t += lanes) {")
    w("        const int k = t / (NW + NWX + NS), e = t - k * (NW + NWX + NS);")
    w("        const double* Sk = I.gm.scratch + (int64_t)k * NCOO;")
    w("        const double* Sn = Sk + NCOO;   // the next stage's scratch (k + 1 < H)")
    w("        const bool next = k + 1 < I.H;")
    w("        if (e < NW) {")
    w("            if (!full) continue;")
    w("            double acc = 0.0;")
    w("            for (int q = RW_PTR[e]; q < RW_PTR[e + 1]; ++q) acc += Sk[RW_IDX[q]];")
    w("            if (next)")
    w("                for (int q = RWN_PTR[e]; q < RWN_PTR[e + 1]; ++q) acc += Sn[RWN_IDX[q]];")
    w("            I.wv[woff(k) + e] = acc;")
    w("        } else if (e < NW + NWX) {")
    w("            if (!full || k == 0) continue;")
    w("            double acc = 0.0;")
    w("            for (int q = RX_PTR[e - NW]; q < RX_PTR[e - NW + 1]; ++q) acc += Sk[RX_IDX[q]];")
    w("            I.wv[woff(k) + e] = acc;")
    w("        } else {")
    w("            const int v = e - NW - NWX;")
    w("            if (full) {")
    w("                double acc = 0.0;")
    w("                for (int q = RG_PTR[v]; q < RG_PTR[v + 1]; ++q) acc += Sk[RG_IDX[q]];")
    w("                if (next)")
    w("                    for (int q = RGN_PTR[v]; q < RGN_PTR[v + 1]; ++q) acc += Sn[RGN_IDX[q]];")
    w("                I.grad[(int64_t)k * NS + v] = acc;")
    w("            }")
    w("            double f = 0.0;")
    w("            for (int q = RF_PTR[v]; q < RF_PTR[v + 1]; ++q) f += Sk[RF_IDX[q]];")
    w("            I.fterm[(int64_t)k * NS + v] = f;")
    w("        }")
    w("    }")
    w("}")
    w("")
    # cold-start guess: the measured state and the last control
    w("extern \"C\" __global__ void __launch_bounds__(kBlock)")
    w("nmpc_stage_guess(const InstPtrs* __restrict__ Ia, Space sp) {")
    w("    int lb;")
    w("    const InstPtrs& I = Ia[block_inst(sp, lb)];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG) return;")
    w("    const int t = lb * kBlock + threadIdx.x;")
    w("    if (t >= I.n) return;")
    w("    const int j = t % NS;")
    w("    double v = 0.0;")
    w("    if (j < NX) {")
    w("        v = I.x0[j];")
    w("    } else if (j < NX + NU) {")
    w("        v = I.uprev[j - NX];")
    if m.guesses:
        w("    } else {")
        w("        const int i = GA_I[j - NX - NU];")
        w("        switch (GA_P[j - NX - NU]) {")
        for gi, gp in enumerate(m.guesses):
            names = {"dt": "I.gm.dt"}
            if gp.nx0:
                names["sx0"] = f"I.x0[G{gi}_X[i * {gp.nx0} + {{j}}]]"
            if gp.nup:
                names["sup"] = f"I.uprev[G{gi}_U[i * {gp.nup} + {{j}}]]"
            if gp.ndata:
                names["sd"] = f"G{gi}_D[i * {gp.ndata} + {{j}}]"
            em = _Emitter(None, names, indent=4)
            val = em.val(gp.expr)
            w(f"            case {gi}: {{")
            out.extend(em.lines)
            w(f"                v = {val};")
            w("                break;")
            w("            }")
        w("            default: break;")
        w("        }")
    w("    }")
    w("    (void)v;")
    w("    I.y[t] = v;")
    w("}")
    w("")
    # parameter contractions (instance 0)
    objs = [(pi, dd) for pi, dd in enumerate(ders) if dd.pat.kind == "obj"]

    def contraction(dd, s, with_prev=True):
        """so d(term)/ds - sum over the variables the term reads (its slots,
        and with_prev the previous stage's controls) of w_var d2(term)/(dvar ds)."""
        dfs = diff(dd.pat.expr, s)
        acc = mul(sym("so"), dfs)
        for j in range(dd.pat.nv):
            d2 = diff(dfs, sym("sv", j))
            if not is_const(d2, 0.0):
                acc = add(acc, neg(mul(sym("w", j), d2)))
        for b in range(dd.pat.npu if with_prev else 0):
            d2 = diff(dfs, sym("spu", b))
            if not is_const(d2, 0.0):
                acc = add(acc, neg(mul(sym("wp", b), d2)))
        return acc

    def obj_names(pi, dd):
        names = {"sv": f"V[P{pi}_V[i * {dd.pat.nv} + {{j}}]]", "dt": "DT", "tr": "TR", "so": "so",
                 "w": f"I.adj_w[(int64_t)k * NS + P{pi}_V[i * {dd.pat.nv} + {{j}}]]"}
        if dd.pat.ndata:
            names["sd"] = f"P{pi}_D[i * {dd.pat.ndata} + {{j}}]"
        if dd.pat.nsp:
            names["ssp"] = f"SP[P{pi}_SP[i * {dd.pat.nsp} + {{j}}]]"
        if dd.pat.npu:
            pu = f"P{pi}_PU[i * {dd.pat.npu} + {{j}}]"
            names["spu"] = f"(k > 0 ? I.y[(int64_t)(k - 1) * NS + NX + {pu}] : I.uprev[{pu}])"
            names["wp"] = f"(k > 0 ? I.adj_w[(int64_t)(k - 1) * NS + NX + {pu}] : 0.0)"
        return names

    w("// Parameter contractions of the sensitivity solve (instance 0):")
    w("// out = [x0 (nx) | setpoint (nsp) | trajectory (H or 0) | last control (nu)].")
    w("extern \"C\" __global__ void __launch_bounds__(kBlock) nmpc_stage_adj(const InstPtrs* __restrict__ Ia) {")
    w("    const InstPtrs& I = Ia[0];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG) return;")
    w("    const int q = blockIdx.x * kBlock + threadIdx.x;")
    w("    const int ntr = I.ntr;")
    w("    const double so = I.adj_seed[I.nu];")
    w("    const double* SP = I.setp;")
    w("    const double DT = I.gm.dt;")
    w("    double* out = I.adj_out;")
    w("    (void)so; (void)SP; (void)DT;")
    w("    if (q < NX) {")
    w("        // x0 enters the first stage's state rows: - sum_rows coefficient * multiplier")
    w("        double acc = 0.0;")
    w("        for (int e = XR_PTR[q]; e < XR_PTR[q + 1]; ++e) acc -= XR_COEF[e] * I.adj_lam[XR_ROW[e]];")
    w("        out[q] = acc;")
    w("        return;")
    w("    }")
    w("    if (q < NX + NSP) {")
    w("        const int jsp = q - NX;")
    w("        double acc = 0.0;")
    w("        for (int k = 0; k < I.H; ++k) {")
    w("            const double* V = I.y + (int64_t)k * NS;")
    w("            const double TR = ntr > 0 ? I.zF[k] : 0.0;")
    w("            (void)V; (void)TR;")
    for pi, dd in objs:
        for slot in range(dd.pat.nsp):
            e = contraction(dd, sym("ssp", slot))
            if is_const(e, 0.0):
                continue
            w(f"            for (int e = P{pi}_S{slot}_PTR[jsp]; e < P{pi}_S{slot}_PTR[jsp + 1]; ++e) {{")
            w(f"                const int i = P{pi}_S{slot}_IDX[e];")
            em = _Emitter(None, obj_names(pi, dd), indent=4)
            v = em.val(e)
            out.extend(em.lines)
            w(f"                acc += {v};")
            w("            }")
    w("        }")
    w("        out[q] = acc;")
    w("        return;")
    w("    }")
    w("    if (q < NX + NSP + ntr) {")
    w("        const int k = q - NX - NSP;")
    w("        const double* V = I.y + (int64_t)k * NS;")
    w("        const double TR = I.zF[k];")
    w("        const int mc = I.mc;")
    w("        const double* om = I.om;")
    w("        (void)V; (void)TR; (void)mc; (void)om;")
    w("        double acc = 0.0;")
    # rows reading the trajectory: - al_r dc_r/dtr - sum_j w_j lam_r d2c_r/(dv_j dtr)
    for pi, dd in enumerate(ders):
        pat = dd.pat
        if pat.kind == "obj" or "tr" not in _kinds(pat.expr):
            continue
        dcs = diff(pat.expr, sym("tr"))
        if is_const(dcs, 0.0):
            continue
        acc_e = neg(mul(sym("al"), dcs))
        for j in range(pat.nv):
            d2 = diff(dcs, sym("sv", j))
            if not is_const(d2, 0.0):
                acc_e = add(acc_e, neg(mul(mul(sym("w", j), sym("lam")), d2)))
        names = {"sv": f"V[P{pi}_V[i * {pat.nv} + {{j}}]]", "dt": "DT", "tr": "TR",
                 "w": f"I.adj_w[(int64_t)k * NS + P{pi}_V[i * {pat.nv} + {{j}}]]"}
        if pat.ndata:
            names["sd"] = f"P{pi}_D[i * {pat.ndata} + {{j}}]"
        if pat.kind == "ineq":
            names["lam"] = "om[2 * mc + r]"
            names["al"] = "I.adj_lam[mc + r]"
            rexpr = f"k * ND + P{pi}_T[i]"
        else:
            names["lam"] = "(om[r] - om[mc + r])"
            names["al"] = "I.adj_lam[r]"
            rexpr = f"k * RPS + P{pi}_T[i]"
        w(f"        for (int i = 0; i < {len(pat.instances)}; ++i) {{")
        w(f"            const int r = {rexpr};")
        em = _Emitter(None, names, indent=3)
        v = em.val(acc_e)
        out.extend(em.lines)
        w(f"            acc += {v};")
        w("        }")
    for pi, dd in objs:
        e = contraction(dd, sym("tr"))
        if is_const(e, 0.0):
            continue
        w(f"        for (int i = 0; i < {len(dd.pat.instances)}; ++i) {{")
        em = _Emitter(None, obj_names(pi, dd), indent=3)
        v = em.val(e)
        out.extend(em.lines)
        w(f"            acc += {v};")
        w("        }")
    w("        out[q] = acc;")
    w("        return;")
    w("    }")
    w("    if (q < NX + NSP + ntr + NU) {")
    w("        // the last control enters the first stage's terms in previous-control slots")
    w("        const int bq = q - NX - NSP - ntr, k = 0;")
    w("        const double* V = I.y;")
    w("        const double TR = ntr > 0 ? I.zF[0] : 0.0;")
    w("        (void)V; (void)TR; (void)bq; (void)k;")
    w("        double acc = 0.0;")
    for pi, dd in objs:
        for slot in range(dd.pat.npu):
            e = contraction(dd, sym("spu", slot), with_prev=False)
            if is_const(e, 0.0):
                continue
            w(f"        for (int i = 0; i < {len(dd.pat.instances)}; ++i) {{")
            w(f"            if (P{pi}_PU[i * {dd.pat.npu} + {slot}] != bq) continue;")
            em = _Emitter(None, obj_names(pi, dd), indent=3)
            v = em.val(e)
            out.extend(em.lines)
            w(f"            acc += {v};")
            w("        }")
    w("        out[q] = acc;")
    w("    }")
    w("}")
    return "\n".join(out) + "\n"


def generate(m: PatternModel) -> GeneratedModel:
    if not m.patterns:
        raise ValueError(f"{m.name}: no patterns")
    ders = [_derive_pattern(p) for p in m.patterns]
    for dd in ders:
        for inst in dd.pat.instances:
            if dd.pat.kind == "obj":
                vs = [int(v) for v in inst["vars"]]
                if len(vs) != dd.pat.nv or len(set(vs)) != len(vs) or not all(0 <= v < m.ns for v in vs):
                    raise ValueError("objective instance: variable slots must be distinct stage variables")
                if len(inst.get("sps", [])) != dd.pat.nsp or not all(0 <= s < m.n_setpoint for s in inst.get("sps", [])):
                    raise ValueError("objective instance: wrong setpoint slots")
                if len(inst.get("data", [])) != dd.pat.ndata:
                    raise ValueError("objective instance: wrong number of data values")
                pus = [int(b) for b in inst.get("pus", [])]
                if len(pus) != dd.pat.npu or len(set(pus)) != len(pus) or not all(0 <= b < m.nu for b in pus):
                    raise ValueError("objective instance: previous-control slots must be distinct controls")
    if any("tr" in _kinds(d.pat.expr) for d in ders):
        m.uses_traj = True
    seen = set()
    for gp in m.guesses:
        bad = _kinds(gp.expr) - {"sx0", "sup", "sd", "dt"}
        if bad:
            raise ValueError(f"a guess pattern uses {sorted(bad)}")
        for inst in gp.instances:
            t = int(inst["target"])
            if not m.nx + m.nu <= t < m.ns or t in seen:
                raise ValueError(f"guess of variable {t}: not an algebraic variable, or guessed twice")
            seen.add(t)
            if (len(inst.get("x0s", [])) != gp.nx0 or len(inst.get("ups", [])) != gp.nup
                    or len(inst.get("data", [])) != gp.ndata
                    or not all(0 <= q < m.nx for q in inst.get("x0s", []))
                    or not all(0 <= q < m.nu for q in inst.get("ups", []))):
                raise ValueError(f"guess of variable {t}: wrong slots")
    st = _structure(m, ders)
    body = _source(m, ders, st, 0)
    tag = _tag(hashlib.sha256(body.encode() + _header_text()).hexdigest())
    g = GeneratedModel(
        name=m.name, nx=m.nx, nu=m.nu, na=m.na, n_alg_rows=st["n_alg"], n_setpoint=m.n_setpoint,
        uses_traj=m.uses_traj,
        row_ptr=np.array(st["row_ptr"], dtype=np.int32), row_cols=np.array(st["row_cols"], dtype=np.int32),
        prev_ptr=np.array(st["prev_ptr"], dtype=np.int32), prev_cols=np.array(st["prev_cols"], dtype=np.int32),
        prev_coef=np.array(st["prev_coef"], dtype=np.float64),
        ineq_ptr=np.array(st["ineq_ptr"], dtype=np.int32), ineq_cols=np.array(st["ineq_cols"], dtype=np.int32),
        w_rows=np.array([a for a, _ in st["wlist"]], dtype=np.int32),
        w_cols=np.array([b for _, b in st["wlist"]], dtype=np.int32),
        wx_rows=np.array([a for a, _ in st["xlist"]], dtype=np.int32),
        wx_cols=np.array([b for _, b in st["xlist"]], dtype=np.int32),
        lb=np.array(m.lb), ub=np.array(m.ub), source=_source(m, ders, st, tag), tag=tag, derived=None)
    g.scratch_per_stage = max(st["ncoo"], 1)
    g.pattern_structure = (ders, st)
    g.pattern_model = m
    return g
