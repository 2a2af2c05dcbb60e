"""Stage-pattern front end (eq. 3): the algebraic pattern of one stage,
differentiated once, generated as HIP kernels the library loads.

A model is written for a generic stage k of a horizon of H stages: its
variables (states, controls, algebraic quantities, in that order), one state
equation per state, extra equality rows and the stage term of the objective.
The expressions may use the stage's variables, the previous stage's states
(the measured x0 at stage 0), a setpoint vector, one trajectory value per
stage and the stage length dt.  Previous states may only enter the state
equations, linearly and with constant coefficients, so that stages couple
only through the Jacobian (the Hessian stays block diagonal) and the
measured state enters the first stage's rows through a constant matrix.

Symbolic differentiation produces every Jacobian entry, Hessian-of-the-
Lagrangian entry, gradient entry and parameter derivative as an expression of
the same symbols, once per model (the pattern repeats over the stages: the
K_SIMD kernels of Section 2).  The generator writes them into one HIP source
with four kernels (value-only and full evaluation in one, cold-start guess,
parameter contractions of the sensitivities), which `compile` turns into a
gfx950 code object; `nmpc.stage_model_structure` hands it with the per-stage
sparsity patterns to the library (family NMPC_FAMILY_STAGE_MODEL).

This module only builds expressions, patterns and source text; it runs no
part of a solve.
"""
from __future__ import annotations

import hashlib
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

FAMILY_STAGE_MODEL = 4
_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
_INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
GEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_gen")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


# ---- expressions ----------------------------------------------------------------------
class Ex:
    """Immutable expression node; structural equality and hashing."""
    __slots__ = ("op", "args", "_h")

    def __init__(self, op, *args):
        self.op = op
        self.args = args
        self._h = hash((op, args))

    def __hash__(self):
        return self._h

    def __eq__(self, other):
        return isinstance(other, Ex) and self._h == other._h and self.op == other.op and self.args == other.args

    def __repr__(self):
        return f"Ex({self.op}, {self.args})"

    def __add__(self, o):
        return add(self, lift(o))

    __radd__ = __add__

    def __sub__(self, o):
        return add(self, neg(lift(o)))

    def __rsub__(self, o):
        return add(lift(o), neg(self))

    def __mul__(self, o):
        return mul(self, lift(o))

    __rmul__ = __mul__

    def __truediv__(self, o):
        return mul(self, power(lift(o), -1.0))

    def __rtruediv__(self, o):
        return mul(lift(o), power(self, -1.0))

    def __neg__(self):
        return neg(self)

    def __pow__(self, p):
        if isinstance(p, Ex):
            raise TypeError("exponents must be numbers")
        return power(self, float(p))


def const(v):
    return Ex("c", float(v))


ZERO, ONE = const(0.0), const(1.0)


def lift(v):
    if isinstance(v, Ex):
        return v
    if isinstance(v, (int, float, np.floating, np.integer)):
        return const(v)
    raise TypeError(f"not an expression: {v!r}")


def is_const(e, v=None):
    return e.op == "c" and (v is None or e.args[0] == v)


def add(a, b):
    if is_const(a) and is_const(b):
        return const(a.args[0] + b.args[0])
    if is_const(a, 0.0):
        return b
    if is_const(b, 0.0):
        return a
    return Ex("+", a, b)


def neg(a):
    if is_const(a):
        return const(-a.args[0])
    if a.op == "neg":
        return a.args[0]
    return Ex("neg", a)


def mul(a, b):
    if is_const(a) and is_const(b):
        return const(a.args[0] * b.args[0])
    if is_const(a, 0.0) or is_const(b, 0.0):
        return ZERO
    if is_const(a, 1.0):
        return b
    if is_const(b, 1.0):
        return a
    if is_const(a, -1.0):
        return neg(b)
    if is_const(b, -1.0):
        return neg(a)
    return Ex("*", a, b)


def power(a, p):
    if p == 0.0:
        return ONE
    if p == 1.0:
        return a
    if is_const(a):
        return const(a.args[0] ** p)
    return Ex("pow", a, p)


def _fn(name):
    def f(a):
        a = lift(a)
        if is_const(a):
            return const(getattr(math, name)(a.args[0]))
        return Ex(name, a)
    f.__name__ = name
    return f


sin, cos, exp, log, sqrt = (_fn(n) for n in ("sin", "cos", "exp", "log", "sqrt"))


def sym(kind, index=0):
    """Leaf symbol.  Kinds: 'x', 'u', 'a' (state, control, algebraic variable
    of the stage), 'px' (previous stage's state), 'sp' (setpoint entry), 'tr'
    (the stage's trajectory value), 'dt', 'x0' and 'up' (measured state and
    last control; guesses only); 'l', 'al' (Lagrange and adjoint multipliers
    of a stage row), 'w' (adjoint solution of a stage variable), 'so'
    (objective seed) appear in generated code only."""
    return Ex("s", kind, int(index))


def diff(e, s, memo=None):
    """d e / d s for a leaf symbol s (memoized per call tree)."""
    memo = {} if memo is None else memo
    got = memo.get(e)
    if got is not None:
        return got
    op = e.op
    if op == "c":
        r = ZERO
    elif op == "s":
        r = ONE if e == s else ZERO
    elif op == "+":
        r = add(diff(e.args[0], s, memo), diff(e.args[1], s, memo))
    elif op == "neg":
        r = neg(diff(e.args[0], s, memo))
    elif op == "*":
        a, b = e.args
        r = add(mul(diff(a, s, memo), b), mul(a, diff(b, s, memo)))
    elif op == "pow":
        a, p = e.args
        da = diff(a, s, memo)
        r = ZERO if is_const(da, 0.0) else mul(mul(const(p), power(a, p - 1.0)), da)
    else:
        a = e.args[0]
        da = diff(a, s, memo)
        if is_const(da, 0.0):
            r = ZERO
        elif op == "sin":
            r = mul(cos(a), da)
        elif op == "cos":
            r = mul(neg(sin(a)), da)
        elif op == "exp":
            r = mul(exp(a), da)
        elif op == "log":
            r = mul(power(a, -1.0), da)
        elif op == "sqrt":
            r = mul(mul(const(0.5), power(a, -0.5)), da)
        else:
            raise ValueError(op)
    memo[e] = r
    return r


def symbols(e, out=None):
    """Leaf symbols of e."""
    out = set() if out is None else out
    stack = [e]
    seen = set()
    while stack:
        x = stack.pop()
        if x in seen:
            continue
        seen.add(x)
        if x.op == "s":
            out.add(x)
        elif x.op != "c":
            stack.extend(a for a in x.args if isinstance(a, Ex))
    return out


def kinds(e):
    return {s.args[0] for s in symbols(e)}


# ---- stage model ------------------------------------------------------------------------
@dataclass
class StageModel:
    """One stage of a transcribed OCP (see the module docstring).  Rows of a
    stage: the state equations in state order, then the equality rows; the
    inequality rows d(stage) <= 0 come after all equality rows."""
    name: str
    n_setpoint: int = 0
    uses_traj: bool = False
    states: list = field(default_factory=list)      # (name, lb, ub)
    controls: list = field(default_factory=list)
    algebraic: list = field(default_factory=list)
    state_rows: dict = field(default_factory=dict)  # state index -> residual
    alg_rows: list = field(default_factory=list)
    ineq_rows: list = field(default_factory=list)
    objective: Ex = ZERO
    guesses: dict = field(default_factory=dict)     # flat variable index -> expression

    def _var(self, group, kind, name, lb, ub):
        group.append((name, float(lb), float(ub)))
        return sym(kind, len(group) - 1)

    def state(self, name, lb=-math.inf, ub=math.inf):
        return self._var(self.states, "x", name, lb, ub)

    def control(self, name, lb=-math.inf, ub=math.inf):
        return self._var(self.controls, "u", name, lb, ub)

    def algebraic_var(self, name, lb=-math.inf, ub=math.inf):
        return self._var(self.algebraic, "a", name, lb, ub)

    @staticmethod
    def prev(x):
        """The previous stage's value of state x (x0 at the first stage)."""
        assert x.op == "s" and x.args[0] == "x"
        return sym("px", x.args[1])

    @staticmethod
    def prev_control(u):
        """The previous stage's value of control u (the last applied control,
        u_prev, at the first stage); objective only."""
        assert u.op == "s" and u.args[0] == "u"
        return sym("pu", u.args[1])

    @staticmethod
    def x0(i):
        return sym("x0", i)

    @staticmethod
    def u_prev(j):
        return sym("up", j)

    def setpoint(self, j):
        if not 0 <= j < self.n_setpoint:
            raise IndexError("setpoint index out of range")
        return sym("sp", j)

    def traj(self):
        self.uses_traj = True
        return sym("tr")

    @property
    def dt(self):
        return sym("dt")

    # equations ---------------------------------------------------------------
    def dynamics(self, x, f):
        """Implicit-Euler state equation x_k - x_{k-1} - dt f(stage k) = 0."""
        self.state_equation(x, x - self.prev(x) - self.dt * lift(f))

    def state_equation(self, x, residual):
        """General state equation of state x; previous states may enter only
        linearly with constant coefficients."""
        assert x.op == "s" and x.args[0] == "x"
        self.state_rows[x.args[1]] = lift(residual)

    def equality(self, e):
        self.alg_rows.append(lift(e))

    def inequality(self, e):
        """A row e(stage) <= 0."""
        self.ineq_rows.append(lift(e))

    def minimize(self, e):
        self.objective = lift(e)

    def guess(self, v, e):
        self.guesses[self.flat(v)] = lift(e)

    # sizes and indexing -----------------------------------------------------------
    @property
    def nx(self):
        return len(self.states)

    @property
    def nu(self):
        return len(self.controls)

    @property
    def ns(self):
        return len(self.states) + len(self.controls) + len(self.algebraic)

    @property
    def rps(self):
        return self.nx + len(self.alg_rows)

    @property
    def nd(self):
        return len(self.ineq_rows)

    def flat(self, v):
        kind, j = v.args
        return {"x": 0, "u": self.nx, "a": self.nx + self.nu}[kind] + j

    def var(self, j):
        """Symbol of flat stage variable j."""
        if j < self.nx:
            return sym("x", j)
        if j < self.nx + self.nu:
            return sym("u", j - self.nx)
        return sym("a", j - self.nx - self.nu)

    def bounds(self):
        allv = self.states + self.controls + self.algebraic
        return np.array([b[1] for b in allv]), np.array([b[2] for b in allv])

    def rows(self):
        missing = set(range(self.nx)) - set(self.state_rows)
        if missing:
            raise ValueError(f"{self.name}: states without an equation: {sorted(missing)}")
        return [self.state_rows[i] for i in range(self.nx)] + list(self.alg_rows)


# ---- derivation -----------------------------------------------------------------------------
@dataclass
class Derived:
    """Everything the kernels compute, as expressions, plus the patterns.
    Symbols besides the stage's own: 'l' / 'ld' (multipliers of the stage's
    equality / inequality rows), 'pu' (previous stage's controls)."""
    model: StageModel
    rows: list            # residual of each equality row
    jcols: list           # own-stage columns of each equality row (ascending)
    jexpr: list           # d row / d v for those columns
    pcols: list           # previous-stage state columns of each state row (ascending)
    pcoef: list           # their constant coefficients
    drows: list           # inequality rows
    dcols: list
    dexpr: list
    grad: list            # d phi / d v_j
    gnext: list           # d phi / d pu_j: the next stage's term in control j's gradient
    wslots: list          # (a, b), a >= b: per-stage lower Hessian pattern
    wexpr: list           # its value from this stage's functions
    wnext: list           # its value from the next stage's objective (pu, pu), else ZERO
    xslots: list          # (a, b): the stage's variable a with the previous stage's control b
    xexpr: list
    adj_sp: list          # per setpoint entry: contribution of one stage
    adj_tr: Ex            # contribution of one stage to its trajectory value
    adj_up: list          # per control: the first stage's contribution to d/du_prev
    guess: list           # per flat variable


_ALLOWED = {
    "row": {"x", "u", "a", "px", "sp", "tr", "dt"},
    "alg": {"x", "u", "a", "sp", "tr", "dt"},
    "obj": {"x", "u", "a", "pu", "sp", "tr", "dt"},
    "guess": {"x0", "up", "sp", "tr", "dt"},
}


def derive(m: StageModel) -> Derived:
    rows = m.rows()
    for r, e in enumerate(rows):
        bad = kinds(e) - _ALLOWED["row" if r < m.nx else "alg"]
        if bad:
            raise ValueError(f"{m.name}: row {r} uses {sorted(bad)}")
    for r, e in enumerate(m.ineq_rows):
        bad = kinds(e) - _ALLOWED["alg"]
        if bad:
            raise ValueError(f"{m.name}: inequality row {r} uses {sorted(bad)}")
    bad = kinds(m.objective) - _ALLOWED["obj"]
    if bad:
        raise ValueError(f"{m.name}: objective uses {sorted(bad)}")
    V = [m.var(j) for j in range(m.ns)]
    PU = [sym("pu", j) for j in range(m.nu)]
    memo = {}

    def d1(e, s):
        return diff(e, s, memo.setdefault(s, {}))

    def own_vars(e):
        return sorted(m.flat(s) for s in symbols(e) if s.args[0] in ("x", "u", "a"))

    def jac(e):
        cols, ex = [], []
        for j in own_vars(e):
            d = d1(e, V[j])
            if not is_const(d, 0.0):
                cols.append(j)
                ex.append(d)
        return cols, ex

    jcols, jexpr, pcols, pcoef = [], [], [], []
    for r, e in enumerate(rows):
        cols, ex = jac(e)
        if r < m.nx and r not in cols:
            raise ValueError(f"{m.name}: state row {r} does not depend on its own state")
        jcols.append(cols)
        jexpr.append(ex)
        pc, pk = [], []
        if r < m.nx:
            for i in range(m.nx):
                d = diff(e, sym("px", i))
                if is_const(d, 0.0):
                    continue
                if not is_const(d):
                    raise ValueError(f"{m.name}: row {r} is not linear in the previous state {i}")
                pc.append(i)
                pk.append(d.args[0])
        pcols.append(pc)
        pcoef.append(pk)
    dcols, dexpr = [], []
    for e in m.ineq_rows:
        cols, ex = jac(e)
        dcols.append(cols)
        dexpr.append(ex)
    in_obj = set(own_vars(m.objective))
    grad = [d1(m.objective, v) if j in in_obj else ZERO for j, v in enumerate(V)]
    gpu = [d1(m.objective, s) for s in PU]
    gnext = [ZERO] * m.ns
    for j in range(m.nu):
        gnext[m.nx + j] = gpu[j]
    # Hessian of the Lagrangian f + sum_r l_r c_r + sum_r ld_r d_r
    # rows holding both columns of each lower pair, in row order
    pair_rows = {}
    for kind, cols_of, ex_of in (("l", jcols, jexpr), ("ld", dcols, dexpr)):
        for r, cols in enumerate(cols_of):
            for ia, a in enumerate(cols):
                for b in cols[:ia + 1]:
                    pair_rows.setdefault((a, b), []).append((kind, r, ex_of[r][ia]))
    obj_vars = in_obj
    wslots, wexpr, wnext = [], [], []
    for a in range(m.ns):
        for b in range(a + 1):
            acc = diff(grad[a], V[b]) if (a in obj_vars and b in obj_vars) else ZERO
            for kind, r, ea in pair_rows.get((a, b), ()):
                d2 = diff(ea, V[b])
                if not is_const(d2, 0.0):
                    acc = add(acc, mul(sym(kind, r), d2))
            nxt = ZERO
            if m.nx <= b <= a < m.nx + m.nu:
                nxt = diff(gpu[a - m.nx], PU[b - m.nx])
            if not (is_const(acc, 0.0) and is_const(nxt, 0.0)):
                wslots.append((a, b))
                wexpr.append(acc)
                wnext.append(nxt)
    xslots, xexpr = [], []
    for a in range(m.ns):
        for b in range(m.nu):
            d2 = diff(grad[a], PU[b])
            if not is_const(d2, 0.0):
                xslots.append((a, b))
                xexpr.append(d2)

    # parameter contraction of one stage for a parameter symbol s:
    #   - sum_v w_v d2L/dv ds - sum_b wp_b d2f/dpu_b ds - sum_r al_r dc_r/ds + so df/ds
    # (wp: the previous stage's control entries of w; not at the first stage)
    def contraction(s):
        dfs = diff(m.objective, s)
        acc = mul(sym("so"), dfs)
        dLs = dfs
        for r, e in enumerate(rows):
            dcs = diff(e, s)
            if not is_const(dcs, 0.0):
                acc = add(acc, neg(mul(sym("al", r), dcs)))
                dLs = add(dLs, mul(sym("l", r), dcs))
        for r, e in enumerate(m.ineq_rows):
            dds = diff(e, s)
            if not is_const(dds, 0.0):
                acc = add(acc, neg(mul(sym("ald", r), dds)))
                dLs = add(dLs, mul(sym("ld", r), dds))
        for j, v in enumerate(V):
            d2 = diff(dLs, v)
            if not is_const(d2, 0.0):
                acc = add(acc, neg(mul(sym("w", j), d2)))
        for b, pu in enumerate(PU):
            d2 = diff(dfs, pu)
            if not is_const(d2, 0.0):
                acc = add(acc, neg(mul(sym("wp", b), d2)))
        return acc

    adj_sp = [contraction(sym("sp", j)) for j in range(m.n_setpoint)]
    adj_tr = contraction(sym("tr"))
    # u_prev enters the first stage's objective only (as pu)
    adj_up = []
    for b in range(m.nu):
        acc = mul(sym("so"), gpu[b])
        for j, v in enumerate(V):
            d2 = diff(gpu[b], v)
            if not is_const(d2, 0.0):
                acc = add(acc, neg(mul(sym("w", j), d2)))
        adj_up.append(acc)
    guess = []
    for j in range(m.ns):
        g = m.guesses.get(j)
        if g is None:
            g = sym("x0", j) if j < m.nx else (sym("up", j - m.nx) if j < m.nx + m.nu else ZERO)
        bad = kinds(g) - _ALLOWED["guess"]
        if bad:
            raise ValueError(f"{m.name}: guess of variable {j} uses {sorted(bad)}")
        guess.append(g)
    return Derived(m, rows, jcols, jexpr, pcols, pcoef, list(m.ineq_rows), dcols, dexpr, grad, gnext, wslots,
                   wexpr, wnext, xslots, xexpr, adj_sp, adj_tr, adj_up, guess)


# ---- C emission ----------------------------------------------------------------------------------
class _Emitter:
    """SSA emission with common-subexpression reuse across nested scopes.
    `names` maps symbol kinds to C text (format field {j}); the stage's own
    variables read from the array named `vname`."""

    def __init__(self, m: StageModel, names, vname="V", indent=2):
        self.m = m
        self.names = names
        self.vname = vname
        self.scopes = [{}]
        self.lines = []
        self.n = 0
        self.indent = indent
        self.prefix = "t"

    def push(self):
        self.scopes.append({})

    def pop(self):
        self.scopes.pop()

    def line(self, text):
        self.lines.append("    " * self.indent + text)

    def leaf(self, e):
        kind, j = e.args
        if kind in ("x", "u", "a"):
            off = {"x": 0, "u": self.m.nx, "a": self.m.nx + self.m.nu}[kind]
            return f"{self.vname}[{off + j}]"
        fmt = self.names.get(kind)
        if fmt is None:
            raise ValueError(f"symbol {kind} not available here")
        return fmt.format(j=j)

    def val(self, e):
        if e.op == "c":
            v = e.args[0]
            return f"({v!r})" if v < 0 else repr(v)
        if e.op == "s":
            return self.leaf(e)
        for sc in reversed(self.scopes):
            if e in sc:
                return sc[e]
        op = e.op
        if op == "+":
            text = f"{self.val(e.args[0])} + {self.val(e.args[1])}"
        elif op == "neg":
            text = f"-{self.val(e.args[0])}"
        elif op == "*":
            text = f"{self.val(e.args[0])} * {self.val(e.args[1])}"
        elif op == "pow":
            a, p = e.args
            s = self.val(a)
            if p == 2.0:
                text = f"{s} * {s}"
            elif p == -1.0:
                text = f"1.0 / {s}"
            elif p == 3.0:
                text = f"{s} * {s} * {s}"
            elif p == 0.5:
                text = f"sqrt({s})"
            elif p == -2.0:
                text = f"1.0 / ({s} * {s})"
            else:
                text = f"pow({s}, {p!r})"
        else:
            text = f"{op}({self.val(e.args[0])})"
        name = f"{self.prefix}{self.n}"
        self.n += 1
        self.line(f"const double {name} = {text};")
        self.scopes[-1][e] = name
        return name


def _tag(src_hash: str) -> int:
    return int(src_hash[:15], 16)


_EVAL_NAMES = {"px": "P[{j}]", "pu": "PU[{j}]", "sp": "SP[{j}]", "tr": "TR", "dt": "DT",
               "l": "(om[row0 + {j}] - om[mc + row0 + {j}])", "ld": "om[2 * mc + drow0 + {j}]"}
# the next stage's objective seen from this stage: its previous controls are ours
_NEXT_NAMES = {"pu": "V[NX + {j}]", "sp": "SP[{j}]", "tr": "TR1", "dt": "DT"}


def _source(d: Derived, tag: int) -> str:
    m = d.model
    ns, nx, nu, rps, nd = m.ns, m.nx, m.nu, m.rps, m.nd
    lanes = max(ns, rps, nd, 1)
    nwo, nwx = len(d.wslots), len(d.xslots)
    has_next = any(not is_const(e, 0.0) for e in d.gnext) or any(not is_const(e, 0.0) for e in d.wnext)
    out = []
    w = out.append
    w(f"// Kernels of the stage model '{m.name}', written by the stage-pattern front end.")
    w("#include \"kernels.h\"")
    w("using namespace nmpc;")
    w("namespace {")
    w(f"constexpr int NS = {ns}, NX = {nx}, NU = {nu}, RPS = {rps}, ND = {nd}, NWO = {nwo}, NWX = {nwx}, "
      f"LANES = {lanes}, NSP = {m.n_setpoint};")
    w(f"constexpr unsigned long long TAG = {tag}ULL;")
    w("// Hessian slots of stage k: its own NWO, then (k > 0) NWX with the previous stage's controls")
    w("__device__ inline int64_t woff(int k) { return k == 0 ? 0 : NWO + (int64_t)(k - 1) * (NWO + NWX); }")
    w("}  // namespace")
    w("")
    w("// descriptor layout these kernels were built against (checked at load)")
    w("extern \"C\" __device__ unsigned int nmpc_stage_abi = kStageAbi;")
    w("")
    w("extern \"C\" __global__ void __launch_bounds__(kBlock)")
    w("nmpc_stage_eval(const InstPtrs* __restrict__ Ia, Space sp, int src, int pred, int full) {")
    w("    int lb;")
    w("    const InstPtrs& I = Ia[block_inst(sp, lb)];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG || !ctl_active(I.ctl, pred)) return;")
    w("    const int t = lb * kBlock + threadIdx.x;")
    w("    if (t >= I.H * LANES) return;")
    w("    // lane-major over stages: the lanes of a wavefront take the same case")
    w("    const int j = t / I.H, k = t - j * I.H;")
    w("    const double* __restrict__ y = src == kSrcIter ? I.y : I.yt;")
    w("    const double* __restrict__ om = src == kSrcUser ? I.dom : I.om;")
    w("    const double* V = y + (int64_t)k * NS;")
    w("    const double* P = k > 0 ? y + (int64_t)(k - 1) * NS : I.x0;")
    w("    const double* PU = k > 0 ? y + (int64_t)(k - 1) * NS + NX : I.uprev;")
    w("    const bool next = k + 1 < I.H;")
    w("    const double* V1 = next ? y + (int64_t)(k + 1) * NS : V;")
    w("    const double* SP = I.setp;")
    w("    const double TR = I.ntr > 0 ? I.zF[k] : 0.0;")
    w("    const double TR1 = I.ntr > 0 && next ? I.zF[k + 1] : 0.0;")
    w("    const double DT = I.gm.dt;")
    w("    const int row0 = k * RPS, drow0 = k * ND, mc = I.mc;")
    w("    double* wv = I.wv + woff(k);")
    w("    (void)V; (void)P; (void)PU; (void)V1; (void)SP; (void)TR; (void)TR1; (void)DT; (void)om; (void)mc;")
    w("    (void)wv; (void)row0; (void)drow0;")
    w("    switch (j) {")
    nslots = nwo + nwx
    slot_lane = {}
    for s_ in range(nslots):
        slot_lane.setdefault(s_ % lanes, []).append(s_)
    for j in range(lanes):
        em = _Emitter(m, _EVAL_NAMES)
        em.line(f"case {j}: {{")
        em.indent += 1
        if j < rps:
            em.line(f"I.c[row0 + {j}] = {em.val(d.rows[j])};")
        if j < nd:
            em.line(f"I.d[drow0 + {j}] = {em.val(d.drows[j])};")
        if j < ns:
            em.line(f"I.fterm[(int64_t)k * NS + {j}] = {em.val(m.objective) if j == 0 else '0.0'};")
        em.line("if (full) {")
        em.indent += 1
        em.push()
        if j < rps:
            em.line(f"double* jr = I.jv + I.jptr[row0 + {j}];")
            if d.pcols[j]:
                em.line("int q = 0;")
                em.line("if (k > 0) {")
                for c in d.pcoef[j]:
                    em.line(f"    jr[q++] = {c!r};")
                em.line("}")
                for e in d.jexpr[j]:
                    em.line(f"jr[q++] = {em.val(e)};")
            else:
                for q, e in enumerate(d.jexpr[j]):
                    em.line(f"jr[{q}] = {em.val(e)};")
        if j < nd:
            em.line(f"double* jd = I.jv + I.jptr[mc + drow0 + {j}];")
            for q, e in enumerate(d.dexpr[j]):
                em.line(f"jd[{q}] = {em.val(e)};")
        if j < ns:
            em.line(f"double g = {em.val(d.grad[j])};")
        mine = slot_lane.get(j, [])
        for s_ in mine:
            if s_ < nwo:
                em.line(f"double w{s_} = {em.val(d.wexpr[s_])};")
        if has_next and ((j < ns and not is_const(d.gnext[j], 0.0)) or
                         any(s_ < nwo and not is_const(d.wnext[s_], 0.0) for s_ in mine)):
            # the next stage's objective term in this stage's controls
            nx_em = _Emitter(m, _NEXT_NAMES, vname="V1", indent=em.indent + 1)
            nx_em.prefix = "n"
            em.line("if (next) {")
            body = []
            if j < ns and not is_const(d.gnext[j], 0.0):
                body.append(f"g += {nx_em.val(d.gnext[j])};")
            for s_ in mine:
                if s_ < nwo and not is_const(d.wnext[s_], 0.0):
                    body.append(f"w{s_} += {nx_em.val(d.wnext[s_])};")
            em.lines.extend(nx_em.lines)
            for b in body:
                em.line("    " + b)
            em.line("}")
        if j < ns:
            em.line(f"I.grad[(int64_t)k * NS + {j}] = g;")
        for s_ in mine:
            if s_ < nwo:
                em.line(f"wv[{s_}] = w{s_};")
        cross = [s_ for s_ in mine if s_ >= nwo]
        if cross:
            em.line("if (k > 0) {")
            em.push()
            em.indent += 1
            for s_ in cross:
                em.line(f"wv[{s_}] = {em.val(d.xexpr[s_ - nwo])};")
            em.indent -= 1
            em.pop()
            em.line("}")
        em.pop()
        em.indent -= 1
        em.line("}")
        em.line("break;")
        em.indent -= 1
        em.line("}")
        out.extend(em.lines)
    w("        default: break;")
    w("    }")
    w("}")
    w("")
    # cold-start guess
    w("extern \"C\" __global__ void __launch_bounds__(kBlock)")
    w("nmpc_stage_guess(const InstPtrs* __restrict__ Ia, Space sp) {")
    w("    int lb;")
    w("    const InstPtrs& I = Ia[block_inst(sp, lb)];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG) return;")
    w("    const int t = lb * kBlock + threadIdx.x;")
    w("    if (t >= I.n) return;")
    w("    const int j = t / I.H, k = t - j * I.H;")
    w("    const double* SP = I.setp;")
    w("    const double TR = I.ntr > 0 ? I.zF[k] : 0.0;")
    w("    const double DT = I.gm.dt;")
    w("    (void)SP; (void)TR; (void)DT;")
    w("    double v = 0.0;")
    w("    switch (j) {")
    gnames = {"x0": "I.x0[{j}]", "up": "I.uprev[{j}]", "sp": "SP[{j}]", "tr": "TR", "dt": "DT"}
    for j in range(ns):
        em = _Emitter(m, gnames)
        em.line(f"case {j}: {{")
        em.indent += 1
        em.line(f"v = {em.val(d.guess[j])};")
        em.line("break;")
        em.indent -= 1
        em.line("}")
        out.extend(em.lines)
    w("        default: break;")
    w("    }")
    w("    I.y[(int64_t)k * NS + j] = v;")
    w("}")
    w("")
    # parameter contractions (instance 0)
    w("// Parameter contractions of the sensitivity solve (instance 0):")
    w("// out = [x0 (nx) | setpoint (nsp) | trajectory (H or 0) | last control (nu)].")
    w("extern \"C\" __global__ void __launch_bounds__(kBlock) nmpc_stage_adj(const InstPtrs* __restrict__ Ia) {")
    w("    const InstPtrs& I = Ia[0];")
    w("    if (I.family != NMPC_FAMILY_STAGE_MODEL || I.gm.tag != TAG) return;")
    w("    const int q = blockIdx.x * kBlock + threadIdx.x;")
    w("    const int ntr = I.ntr, mc = I.mc;")
    w("    const double so = I.adj_seed[I.nu];")
    w("    const double* om = I.om;")
    w("    const double* SP = I.setp;")
    w("    const double DT = I.gm.dt;")
    w("    double* out = I.adj_out;")
    w("    (void)so; (void)om; (void)SP; (void)DT; (void)mc;")
    w("    if (q < NX) {")
    w("        double acc = 0.0;")
    # x0_j: - sum_i C_ij al_i over the state rows of stage 0
    w("        switch (q) {")
    for jx in range(nx):
        terms = []
        for i in range(nx):
            if jx in d.pcols[i]:
                cij = d.pcoef[i][d.pcols[i].index(jx)]
                terms.append(f"acc -= {cij!r} * I.adj_lam[{i}];")
        w(f"            case {jx}: {{ {' '.join(terms)} break; }}")
    w("            default: break;")
    w("        }")
    w("        out[q] = acc;")
    w("        return;")
    w("    }")
    adj_names = {"sp": "SP[{j}]", "tr": "TR", "dt": "DT", "so": "so", "pu": "PU[{j}]",
                 "l": "(om[row0 + {j}] - om[mc + row0 + {j}])", "ld": "om[2 * mc + drow0 + {j}]",
                 "al": "I.adj_lam[row0 + {j}]", "ald": "I.adj_lam[mc + drow0 + {j}]",
                 "w": "I.adj_w[(int64_t)k * NS + {j}]", "wp": "WP({j})"}

    def stage_body(expr, indent):
        em = _Emitter(m, adj_names, indent=indent)
        v = em.val(expr)
        return em.lines, v

    stage_setup = [
        "const double* V = I.y + (int64_t)k * NS;",
        "const double* PU = k > 0 ? I.y + (int64_t)(k - 1) * NS + NX : I.uprev;",
        "const double TR = ntr > 0 ? I.zF[k] : 0.0;",
        "const int row0 = k * RPS, drow0 = k * ND;",
        "auto WP = [&](int b) { return k > 0 ? I.adj_w[(int64_t)(k - 1) * NS + NX + b] : 0.0; };",
        "(void)V; (void)PU; (void)TR; (void)row0; (void)drow0; (void)WP;",
    ]
    w("    if (q < NX + NSP) {")
    w("        const int jsp = q - NX;")
    w("        double acc = 0.0;")
    w("        for (int k = 0; k < I.H; ++k) {")
    for line in stage_setup:
        w("            " + line)
    w("            switch (jsp) {")
    for jsp, expr in enumerate(d.adj_sp):
        lines, v = stage_body(expr, 5)
        w(f"                case {jsp}: {{")
        out.extend(lines)
        w(f"                    acc += {v};")
        w("                    break;")
        w("                }")
    w("                default: break;")
    w("            }")
    w("        }")
    w("        out[q] = acc;")
    w("        return;")
    w("    }")
    w("    if (q < NX + NSP + ntr) {")
    w("        const int k = q - NX - NSP;")
    for line in stage_setup:
        w("        " + line)
    lines, v = stage_body(d.adj_tr, 2)
    out.extend(lines)
    w(f"        out[q] = {v};")
    w("        return;")
    w("    }")
    w("    if (q < NX + NSP + ntr + NU) {")
    w("        const int k = 0, jup = q - NX - NSP - ntr;")
    for line in stage_setup:
        w("        " + line)
    w("        double acc = 0.0;")
    w("        switch (jup) {")
    for b, expr in enumerate(d.adj_up):
        lines, v = stage_body(expr, 3)
        w(f"            case {b}: {{")
        out.extend(lines)
        w(f"                acc = {v};")
        w("                break;")
        w("            }")
    w("            default: break;")
    w("        }")
    w("        out[q] = acc;")
    w("    }")
    w("}")
    w("")
    return "\n".join(out) + "\n"


# ---- generated model ----------------------------------------------------------------------------
@dataclass
class GeneratedModel:
    """Source, per-stage patterns and bounds of a model; `code` holds the
    compiled code object once `compile` has run."""
    name: str
    nx: int
    nu: int
    na: int
    n_alg_rows: int
    n_setpoint: int
    uses_traj: bool
    row_ptr: np.ndarray
    row_cols: np.ndarray
    prev_ptr: np.ndarray
    prev_cols: np.ndarray
    prev_coef: np.ndarray
    ineq_ptr: np.ndarray
    ineq_cols: np.ndarray
    w_rows: np.ndarray
    w_cols: np.ndarray
    wx_rows: np.ndarray
    wx_cols: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    source: str
    tag: int
    derived: Derived = None
    code: bytes = b""
    path: str = ""
    scratch_per_stage: int = 0   # pattern models: doubles of per-stage scratch the kernels sum

    @property
    def ns(self):
        return self.nx + self.nu + self.na

    @property
    def rps(self):
        return self.nx + self.n_alg_rows


def _header_text():
    parts = []
    for f in sorted(os.listdir(_CSRC)):
        if f.endswith(".h"):
            with open(os.path.join(_CSRC, f), "rb") as fh:
                parts.append(fh.read())
    with open(os.path.join(_INCLUDE, "nmpc.h"), "rb") as fh:
        parts.append(fh.read())
    return b"".join(parts)


def generate(m: StageModel) -> GeneratedModel:
    d = derive(m)
    row_ptr = np.zeros(m.rps + 1, dtype=np.int32)
    prev_ptr = np.zeros(m.rps + 1, dtype=np.int32)
    for r in range(m.rps):
        row_ptr[r + 1] = row_ptr[r] + len(d.jcols[r])
        prev_ptr[r + 1] = prev_ptr[r] + len(d.pcols[r])
    # the tag names the kernels: a hash of the expressions and of the headers
    # that fix the descriptor layout they read
    body = _source(d, 0)
    h = hashlib.sha256(body.encode() + _header_text()).hexdigest()
    tag = _tag(h)
    lb, ub = m.bounds()
    return GeneratedModel(
        name=m.name, nx=m.nx, nu=m.nu, na=len(m.algebraic), n_alg_rows=len(m.alg_rows),
        n_setpoint=m.n_setpoint, uses_traj=m.uses_traj,
        row_ptr=row_ptr, row_cols=np.array([c for cs in d.jcols for c in cs], dtype=np.int32),
        prev_ptr=prev_ptr, prev_cols=np.array([c for cs in d.pcols for c in cs], dtype=np.int32),
        prev_coef=np.array([c for cs in d.pcoef for c in cs], dtype=np.float64),
        ineq_ptr=np.concatenate([[0], np.cumsum([len(c) for c in d.dcols])]).astype(np.int32),
        ineq_cols=np.array([c for cs in d.dcols for c in cs], dtype=np.int32),
        w_rows=np.array([a for a, _ in d.wslots], dtype=np.int32),
        w_cols=np.array([b for _, b in d.wslots], dtype=np.int32),
        wx_rows=np.array([a for a, _ in d.xslots], dtype=np.int32),
        wx_cols=np.array([b for _, b in d.xslots], dtype=np.int32),
        lb=lb, ub=ub, source=_source(d, tag), tag=tag, derived=d)


HIP_FLAGS = ["--genco", "--offload-arch=gfx950", "-O3", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def compile(m: StageModel | GeneratedModel, cache_dir: str = GEN_DIR, force: bool = False) -> GeneratedModel:
    """Generate (if needed) and compile the model's kernels to a gfx950 code
    object, cached under cache_dir by the model's tag."""
    if isinstance(m, GeneratedModel):
        g = m
    elif isinstance(m, StageModel):
        g = generate(m)
    else:                  # index-data pattern models generate themselves
        g = m.generate()
    os.makedirs(cache_dir, exist_ok=True)
    stem = os.path.join(cache_dir, f"{g.name}_{g.tag:015x}")
    src, obj = stem + ".hip", stem + ".hsaco"
    if force or not os.path.exists(obj):
        with open(src, "w") as fh:
            fh.write(g.source)
        tmp = obj + f".{os.getpid()}.tmp"
        cmd = [HIPCC, *HIP_FLAGS, "-I", _CSRC, "-o", tmp, src]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling the kernels of '{g.name}' failed:\n{r.stderr[-4000:]}")
        os.replace(tmp, obj)
    with open(obj, "rb") as fh:
        g.code = fh.read()
    g.path = obj
    return g
