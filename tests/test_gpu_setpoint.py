"""Set-point -> separation on the GPU (many pixels, one launch per round) against the oracle's
approach-curve search, which integrates each steady amplitude to convergence."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_separations_match_oracle(orc):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1109_0334_amd as afm
    from paper_1109_0334_amd import setpoint

    c = W.config("c3")
    m = dict(c["model"], steps_per_cycle=64)
    base = W.full_params(c)
    estar = np.array([0.3e9, 2.0e9, 20e9])
    sp = np.array([0.85, 0.7, 0.55])
    zc = setpoint.separations(afm, m, base, [2], [estar], sp, periods=3000)
    for s in range(3):
        p = base.copy()
        p[2] = estar[s]
        zo = orc.zc_from_setpoint(m, p, sp[s])
        print(f"pixel {s}: E* {estar[s]:.3g} s {sp[s]}: gpu {zc[s]:.15e} oracle {zo:.15e}")
        assert np.isfinite(zo) and abs(zc[s] - zo) < 5e-13
