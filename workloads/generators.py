"""Seeded input generators for the NMPC workloads.

Every random number a workload needs is drawn here, in a fixed order, from
``numpy.random.default_rng(seed)``.  Nothing here evaluates a model or runs any
part of the solver: the generators return plain arrays and constants.

Workload recipe (synthetic stand-ins for the paper's two NMPC case-study
families, Section 4.1 distillation column and Section 4.2 heated plate):

distillation
    ``N`` trays plus condenser and reboiler (``nx = N + 2`` liquid mole
    fractions), controls ``u = (R, V)`` (reflux, boilup), implicit-Euler
    transcription over ``H`` stages of length ``dt``.  Relative volatility
    ``alpha`` is fixed (small case) or drawn ``U(2, 3)`` once per seed.  The
    feed composition trajectory over the horizon is constant 0.5 (small case)
    or ``0.5 + 0.05 sin(t_now + k dt)``.  The initial measured state is a
    smooth composition profile (0.93 at the top, 0.07 at the bottom) plus
    ``N(0, 0.01^2)`` noise, clipped to [0, 1].  After each solve the next
    measurement is the first predicted state plus fresh ``N(0, 0.01^2)``
    noise, clipped to [0, 1]; the noise vectors are pre-drawn here.

plate
    ``G x G`` interior grid, 16 boundary heater segments, ``H`` implicit-Euler
    stages.  Target field is a Gaussian bump with amplitude ``U(0.3, 0.8)``,
    centre ``U(0.3, 0.7)^2`` and width ``U(0.1, 0.25)``; initial field 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class DistillationWorkload:
    name: str
    seed: int
    N: int                  # number of trays (states = N + 2)
    H: int                  # horizon stages
    dt: float
    alpha: float
    F: float                # feed flow
    xD_sp: float            # top (distillate) purity setpoint
    xB_sp: float            # bottom purity setpoint
    rho: float              # control-move penalty
    u_prev0: np.ndarray     # (2,) control applied before the first solve
    x0: np.ndarray          # (N+2,) first measured state
    resolve_noise: np.ndarray  # (n_resolves, N+2) measurement noise per re-solve
    zF_amp: float           # feed composition disturbance amplitude (0 = constant)
    n_resolves: int
    x_lo: float = 0.0
    x_hi: float = 1.0
    u_lo: float = 0.5
    u_hi: float = 5.0
    Hc: int = 0             # control horizon in stages (0: the whole horizon)

    @property
    def nx(self) -> int:
        return self.N + 2

    @property
    def nu(self) -> int:
        return 2

    @property
    def feed_tray(self) -> int:
        return self.N // 2

    def zF(self, solve_index: int) -> np.ndarray:
        """Feed composition over the horizon for the given solve (length H).

        Solve ``r`` starts at ``t_now = r * dt``; stage k (1-based) sees
        ``0.5 + amp * sin(t_now + k * dt)``.
        """
        t_now = solve_index * self.dt
        k = np.arange(1, self.H + 1, dtype=np.float64)
        return 0.5 + self.zF_amp * np.sin(t_now + k * self.dt)

    def next_measurement(self, x1_pred: np.ndarray, solve_index: int) -> np.ndarray:
        """Measurement fed to solve ``solve_index + 1``: predicted x_1 plus noise."""
        x = np.asarray(x1_pred, dtype=np.float64) + self.resolve_noise[solve_index]
        return np.clip(x, self.x_lo, self.x_hi)


def _profile(nx: int) -> np.ndarray:
    i = np.arange(nx, dtype=np.float64)
    return 0.5 + 0.45 * np.tanh(4.0 * (0.5 - i / (nx - 1)))


def distillation_workload(name: str = "small", seed: int = 0, **over) -> DistillationWorkload:
    """Build a distillation workload.

    ``small``: 10 trays, alpha 2.5, horizon 20, dt 0.1, constant feed, 5 re-solves.
    ``medium``: 40 trays, alpha ~ U(2,3), horizon 100, dt 0.05, sinusoidal feed
    composition, 50 re-solves.
    Keyword overrides (N, H, dt, n_resolves, alpha) allow reduced variants for
    tests; random draws keep their order so a seed always yields the same stream.
    """
    rng = np.random.default_rng(seed)
    if name == "small":
        N, H, dt, nres, amp = 10, 20, 0.1, 5, 0.0
        alpha_draw = None
    elif name == "medium":
        N, H, dt, nres, amp = 40, 100, 0.05, 50, 0.05
        alpha_draw = True
    else:
        raise ValueError(f"unknown distillation workload {name!r}")
    N = over.pop("N", N)
    H = over.pop("H", H)
    dt = over.pop("dt", dt)
    nres = over.pop("n_resolves", nres)
    amp = over.pop("zF_amp", amp)
    nx = N + 2
    alpha = float(rng.uniform(2.0, 3.0)) if alpha_draw else 2.5
    alpha = over.pop("alpha", alpha)
    x0 = np.clip(_profile(nx) + rng.normal(0.0, 0.01, nx), 0.0, 1.0)
    noise = rng.normal(0.0, 0.01, (max(nres, 1), nx))
    xD = over.pop("xD_sp", 0.95)
    xB = over.pop("xB_sp", 0.05)
    Hc = over.pop("Hc", 0)
    if over:
        raise TypeError(f"unknown overrides {sorted(over)}")
    return DistillationWorkload(
        name=name, seed=seed, N=N, H=H, dt=dt, alpha=alpha, F=1.0,
        xD_sp=xD, xB_sp=xB, rho=1e-2, u_prev0=np.array([2.0, 2.5]),
        x0=x0, resolve_noise=noise, zF_amp=amp, n_resolves=nres, Hc=Hc)


def batch_distillation_workloads(count: int = 64, base_seed: int = 1000):
    """Ragged batch: trays ~ U{20..60}, horizon ~ U{40..120}, alpha ~ U(2,3),
    setpoints xD ~ U(0.90, 0.98), xB ~ U(0.02, 0.10); instance i uses seed base+i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        N = int(rng.integers(20, 61))
        H = int(rng.integers(40, 121))
        alpha = float(rng.uniform(2.0, 3.0))
        xD = float(rng.uniform(0.90, 0.98))
        xB = float(rng.uniform(0.02, 0.10))
        nx = N + 2
        x0 = np.clip(_profile(nx) + rng.normal(0.0, 0.01, nx), 0.0, 1.0)
        noise = rng.normal(0.0, 0.01, (10, nx))
        out.append(DistillationWorkload(
            name="batch", seed=base_seed + i, N=N, H=H, dt=0.05, alpha=alpha, F=1.0,
            xD_sp=xD, xB_sp=xB, rho=1e-2, u_prev0=np.array([2.0, 2.5]), x0=x0,
            resolve_noise=noise, zF_amp=0.05, n_resolves=10))
    return out


@dataclass
class PlateWorkload:
    name: str
    seed: int
    G: int
    H: int
    dt: float
    n_resolves: int
    target: np.ndarray = field(repr=False)   # (G*G,) row-major (b, a) -> b*G + a
    bump: tuple = (0.0, 0.0, 0.0, 0.0)       # (A, cx, cy, sigma)
    T0: np.ndarray = field(default=None, repr=False)
    T_hi: float = 1.5
    u_lo: float = 0.0
    u_hi: float = 1.0
    n_controls: int = 16


def plate_workload(name: str = "large", seed: int = 0, **over) -> PlateWorkload:
    """Heated plate: ``large`` = 32x32 grid, H 50, dt 0.01, 20 re-solves;
    ``adjoint`` = 64x64 grid, H 100, dt 0.01, 10 re-solves."""
    rng = np.random.default_rng(seed)
    if name == "large":
        G, H, dt, nres = 32, 50, 0.01, 20
    elif name == "adjoint":
        G, H, dt, nres = 64, 100, 0.01, 10
    else:
        raise ValueError(f"unknown plate workload {name!r}")
    G = over.pop("G", G)
    H = over.pop("H", H)
    dt = over.pop("dt", dt)
    nres = over.pop("n_resolves", nres)
    if over:
        raise TypeError(f"unknown overrides {sorted(over)}")
    A = float(rng.uniform(0.3, 0.8))
    cx, cy = (float(v) for v in rng.uniform(0.3, 0.7, 2))
    sig = float(rng.uniform(0.1, 0.25))
    h = 1.0 / (G + 1)
    coord = h * np.arange(1, G + 1)
    X, Y = np.meshgrid(coord, coord)          # X[b, a] = a-th x, Y[b, a] = b-th y
    target = A * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
    return PlateWorkload(name=name, seed=seed, G=G, H=H, dt=dt, n_resolves=nres,
                         target=target.reshape(-1), bump=(A, cx, cy, sig),
                         T0=np.zeros(G * G))


WORKLOADS = {
    "distill_small": lambda seed=0, **kw: distillation_workload("small", seed, **kw),
    "distill_medium": lambda seed=0, **kw: distillation_workload("medium", seed, **kw),
    "plate_large": lambda seed=0, **kw: plate_workload("large", seed, **kw),
    "plate_adjoint": lambda seed=0, **kw: plate_workload("adjoint", seed, **kw),
}


@dataclass
class RefluxWorkload:
    """The distillation case study of Section 4.1 (Table 1): 32 trays, feed on
    tray 17, reflux-ratio control, horizon 180 s of 2 s stages, closed loop
    from t = 0 to 300 s (150 NMPC steps), plant = the model."""
    N: int = 32
    Nf: int = 17
    D: float = 0.2
    F: float = 0.4
    alpha: float = 1.6
    xbar: float = 0.8958
    ubar: float = 2.51459
    xf: float = 0.5
    Ac: float = 0.5
    At: float = 0.25
    Ar: float = 1.0
    w_u: float = 0.1
    dt: float = 2.0
    H: int = 90
    n_steps: int = 150
    x0: np.ndarray = None   # first measured tray compositions (condenser first)
    u_prev0: float = 2.0    # reflux ratio before the first solve


def reflux_workload(**over) -> RefluxWorkload:
    """The case study's parameters.  The paper gives no initial state; the
    loop starts from a linear composition profile, 0.85 at the condenser to
    0.12 at the reboiler, away from the steady state the controller targets."""
    w = RefluxWorkload(**over)
    if w.x0 is None:
        w.x0 = np.linspace(0.85, 0.12, w.N)
    return w


def random_lq(nx, nu, H, seed, spectral_radius=0.95, indefinite=False):
    """Seeded stable (A, B) and SPD weights (Q may be made indefinite)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(nx, nx))
    A *= spectral_radius / max(abs(np.linalg.eigvals(A)))
    B = rng.normal(size=(nx, nu))
    M = rng.normal(size=(nx, nx))
    Q = M @ M.T / nx + 0.1 * np.eye(nx)
    if indefinite:
        Q[0, 0] -= 2.0 * (np.max(np.linalg.eigvalsh(Q)) + 1.0)
    Mr = rng.normal(size=(nu, nu))
    Rw = Mr @ Mr.T / nu + 0.5 * np.eye(nu)
    x0 = rng.normal(size=nx)
    xs = rng.normal(size=nx) * 0.5
    return A, B, Q, Rw, x0, xs


@dataclass
class PlateCaseWorkload:
    """The heated-plate case study of Section 4.2 (Table 2): a 21 x 21 grid on
    [-1, 1]^2 (spacing 0.1 = L), alpha 230, T_b 50, rho 1e-8, q_loss 10, Q >= 50;
    NMPC steps of dt = 0.08 s from t = 0 to 3 s (38 steps), horizon 12 stages
    (0.96 s: the printed 1.0 s is not a multiple of dt), setpoint 58 / 55 / 63
    switching at 0.5 s and 1.5 s, plate initially at T_b (the paper gives no
    T_0), plant = model.  The loss term is read as 5 q_loss (printed 5 q_loss^2;
    see the design notes); the input enters the problem in units of q_scale."""
    n: int = 21
    alpha: float = 230.0
    Tb: float = 50.0
    q_loss: float = 10.0
    loss: float = 50.0
    rho: float = 1e-8
    Q_lo: float = 50.0
    q_scale: float = 1e4
    dt: float = 0.08
    H: int = 12
    n_steps: int = 38
    T0: float = 50.0
    Q_prev0: float = 50.0

    @staticmethod
    def setpoint(t):
        t = np.asarray(t, dtype=np.float64)
        return np.where(t < 0.5, 58.0, np.where(t < 1.5, 55.0, 63.0))

    def traj(self, k):
        """Tracked temperature of the H stages of the solve at step k (t = k dt)."""
        return self.setpoint(self.dt * (k + np.arange(1, self.H + 1)))

    @property
    def nx(self):
        return (self.n - 2) ** 2


def plate_case_workload(**over) -> PlateCaseWorkload:
    return PlateCaseWorkload(**over)

