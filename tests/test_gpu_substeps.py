"""Sub-increments of an increment whose Newton solve does not converge.

On the 256^2 fibre composite (crack-length increments of 2) the 62nd
increment's Newton iterates cycle between four states at any relaxation
alpha in [0.5, 1] (the paper's remedy for developed cracks is alpha < 1);
two increments of 1 converge.  The library retries a failing increment as
two half increments from the committed state, recursively down to
delta_a / 8, each committing its history.  GPU outputs only: the oracle
comparison of the first increments is the increment parity test.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_failing_increment_is_taken_in_sub_increments(monkeypatch):
    from paper_2412_17445_amd import Solver
    from synth import problem_config
    prob = problem_config("fibres2d_256")
    s = Solver.from_problem(prob, precision="fp64")
    s.bootstrap()
    for _ in range(61):
        o = s.step()
        assert o["converged"] and o["newton_iters"] < 20, o
    eps, phi, Hn, E, a = s.get_state()
    fm = np.array([prob.f[0, 0], prob.f[1, 1], np.sqrt(2.0) * prob.f[0, 1]])
    eps_t = eps - fm.reshape((3, 1, 1, 1)) * E

    # without sub-increments the increment fails and the state is rolled back
    monkeypatch.setenv("PFF_SUBSTEPS", "0")
    r = Solver.from_problem(prob, precision="fp64")
    monkeypatch.delenv("PFF_SUBSTEPS")
    r.set_state(eps_t, phi, Hn, E, a, n=61)
    o = r.step()
    assert not o["converged"], o
    _, phi_r, Hn_r, E_r, a_r = r.get_state()
    assert a_r == a and E_r == E
    assert np.array_equal(phi_r, phi) and np.array_equal(Hn_r, Hn)
    r.close()

    # with them (the default) the same increment reaches its target
    o = s.step()
    print(f"increment 62: newton {o['newton_iters']} (all attempts), krylov {o['krylov_iters']}, "
          f"E {o['E']:.6e} (from {E:.6e}), Gamma {o['Gamma']:.6f}", flush=True)
    assert o["converged"] and o["increment"] == 62
    assert abs(o["Gamma"] - (a + prob.delta_a)) <= 1e-8 * (a + prob.delta_a)
    assert abs(o["a"] - (a + prob.delta_a)) <= 1e-12 * (a + prob.delta_a)
    _, _, Hn2, _, _ = s.get_state()
    assert (Hn2 >= Hn).all()                      # the sub-increments committed history
    o = s.step()
    assert o["converged"] and o["increment"] == 63
    s.close()
