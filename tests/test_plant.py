"""The closed-loop plant simulator (paper_2606_04725_amd/plant.py) against
the oracle's transcription: with the model's parameters, one plant step is
the state at which the stage-1 implicit-Euler rows of the oracle's model
vanish.  Runs without a GPU."""
import numpy as np
import pytest

from oracle.distillation import DistillationOCP
from paper_2606_04725_amd.plant import DistillationPlant
from workloads import distillation_workload


@pytest.mark.parametrize("kind,seed", [("small", 0), ("medium", 2)])
def test_plant_step_zeroes_the_models_first_stage(kind, seed):
    w = distillation_workload(kind, seed)
    zF = float(w.zF(0)[0])
    u = np.array([2.3, 2.9])
    plant = DistillationPlant(w.N, w.alpha, w.dt, F=w.F)
    x1 = plant.step(w.x0, u, zF=zF)
    m = DistillationOCP(w.N, 1, w.dt, w.alpha, F=w.F)
    m.set_parameters(x0=w.x0, zF=[zF], u_prev=u)
    y = np.concatenate([x1, u])
    assert np.max(np.abs(m.cons_c(y))) <= 1e-12


def test_mismatched_plant_differs():
    w = distillation_workload("small", 0)
    u = np.array([2.3, 2.9])
    a = DistillationPlant(w.N, w.alpha, w.dt).step(w.x0, u)
    b = DistillationPlant(w.N, 1.08 * w.alpha, w.dt).step(w.x0, u)
    assert np.max(np.abs(a - b)) > 1e-4
