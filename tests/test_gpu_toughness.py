"""Effective toughness of a homogeneous cracked panel (paper Sec. 2.4 eq.
JaviGc, Sec. 5.2), a sanity check against the paper's own result.

The paper loads homogeneous Griffith panels (257^2 voxels, l = 2 voxels)
with a central crack under crack-length control until the crack coalesces
with its periodic image, integrates the macroscopic curve and finds
G_Ceff = 3232.6 for an input Gc = 2700, a ratio of 1.197 (the diffuse crack
dissipates more than Gc per unit length; its Appendix A.1 fits the
amplification of a 1D profile as 1 + 0.298 / (l/h), 1.149 at l = 2h).

Here: 128^2 and 256^2 homogeneous cells, a central crack of a quarter of
the width, l = 2, uniaxial tension across the crack, crack-length
increments of 2 voxel-lengths until the macroscopic stress has fallen below
5% of its peak (the ligament is broken; the elastic energy left is about 1%
of Gc L_g).  G_Ceff = N * integral of Sigma_M : f dE / (L - a0) through
pff_effective_toughness.  Not a parity test (the oracle is far too slow for
these paths): the bar is the band 1.05 < G_Ceff / Gc < 1.35 around the
paper's 1.197.  The test also reports the rise of the crack functional per
unit crack length, (Gamma_end - Gamma_0) / L_g, the dissipation the path
would carry if it balanced energy exactly; the work integral sits a few
percent below it and approaches it as the path is refined.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n", [128, 256])
def test_griffith_panel_effective_toughness(n):
    from paper_2412_17445_amd import Solver, effective_toughness
    from synth.microstructure import line_crack_mask
    a0, Gc, l = n // 4, 1e-3, 2.0
    f = np.zeros((3, 3))
    f[1, 1] = 1.0
    s = Solver((1, n, n), [(1.0, 0.3, Gc)], np.zeros((1, n, n), np.uint8),
               line_crack_mask(n, n, n // 2, (n - a0) // 2, (n + a0) // 2), f, l, delta_a=2.0,
               krylov_rtol=1e-8, precision="fp64")
    gamma0, _ = s.bootstrap()
    E, S, peak = [], [], 0.0
    for _ in range(4 * n):
        out = s.step()
        if not out["converged"]:
            break
        E.append(out["E"])
        S.append(out["sigma_M"])
        peak = max(peak, out["sigma_M"][1])
        if len(E) % 10 == 0:
            print(f"increment {out['increment']}: E {out['E']:.5e} Gamma {out['Gamma']:.3f} "
                  f"Sigma_yy {out['sigma_M'][1]:.4e} newton {out['newton_iters']}", flush=True)
        if out["sigma_M"][1] < 0.05 * peak:
            break
    s.close()
    assert S and S[-1][1] < 0.05 * peak, (len(S), S[-1][1] if S else None, peak)
    work, gceff = effective_toughness(np.array(E), np.array(S), f, volume=n * n, L_g=n - a0)
    ratio = gceff / Gc
    rise = (out["Gamma"] - gamma0) / (n - a0)
    print(f"Griffith panel {n}^2, l = 2: {len(E)} increments, G_Ceff / Gc = {ratio:.4f}, "
          f"Gamma rise per unit length {rise:.4f} (paper Sec. 5.2: 1.197 on 257^2; "
          f"Appendix A.1 fit at l = 2h: 1.149)", flush=True)
    assert 1.05 < ratio < 1.35, ratio
