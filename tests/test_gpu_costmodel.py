"""The measured cost model: calibration on the device, predictions that rank
clearly different pass parameters the way the device does."""

import pytest

from workloads import layered_circuit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import costmodel  # noqa: E402


def test_calibration_costs_are_positive_and_fit():
    cm = costmodel.CostModel("c128", n_cal=22)
    cm.calibrate([(10, 0)])
    tc = cm.tile_costs[(10, 0)]
    assert tc["tile_pass"] > 0 and tc["u"] > 0 and tc["remap"] > 0
    assert cm.fit_residual[(10, 0)] < 0.25
    assert all(v > 0 for k, v in cm.launch_costs.items() if k != "move")


def test_model_orders_clear_choices_like_the_device():
    n = 24
    g = layered_circuit(n, 12, 20100946 + 11)
    cm = costmodel.CostModel("c128", n_cal=22)
    good = dict(k_tile=10, max_swaps=8, pinned=3, perm_exec="relabel", reg_bits=0)
    poor = dict(k_tile=7, max_swaps=1, pinned=0, perm_exec="relabel", reg_bits=0)
    cm.calibrate([(10, 0), (7, 0)])
    pg, _ = cm.predict(g, n, **good)
    pp, _ = cm.predict(g, n, **poor)
    mg = costmodel.measure_ms(g, n, "c128", good)
    mp = costmodel.measure_ms(g, n, "c128", poor)
    assert pg < pp and mg < mp
    # the prediction is within a factor of two of the measurement
    assert 0.5 < pg / mg < 2.0


@pytest.mark.parametrize("perm_exec,r,move", [("move", 1, 2.0), ("relabel", 4, 0.0)])
def test_costed_pass_program_matches_oracle(perm_exec, r, move):
    """A program whose PermuteQubits and gates run on their own were chosen by
    predicted time (qs_compile_costed) computes the circuit: full vector
    against the oracle."""
    import numpy as np

    import oracle as O
    from paper_2010_09746_amd import qsim as Q
    from workloads import config_circuit

    n = 16
    g = config_circuit(2, n=n, layers=12)
    costs = Q.make_pass_costs(1.0, (0.02, 0.03, 0.005), move, (1.0, 1.0, 0.8, 1.1))
    P = Q.Program(g, n, "c128", form="pass", k_tile=10, max_swaps=r, pinned=0 if r == 1 else 3, perm_exec=perm_exec,
                  costs=costs)
    st = P.stats()
    s = Q.State(n, "c128")
    s.run_program(P)
    v = s.to_numpy()
    s.close()
    P.close()
    if perm_exec == "move":
        assert st["n_global"] > 0
    ref = O.run(g, n)
    assert np.abs(v - ref).max() <= 1e-12
    # the same choices when the pass and the launches advance together
    s = Q.State(n, "c128")
    s.run(g, costs=costs, form="pass", k_tile=10, max_swaps=r, pinned=0 if r == 1 else 3, perm_exec=perm_exec)
    w = s.to_numpy()
    s.close()
    assert np.abs(w - ref).max() <= 1e-12
