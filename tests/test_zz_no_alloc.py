"""The photoionisation step without allocation (sweep_ion_step_noalloc, the
library's static scratch word instead of a buffer of the DAG) against
sweep_ion_step on the same inputs, through the C ABI: two calls in a row, the
second on a smaller mesh whose step limit is larger than the first's, so a word
left holding the first call's minimum would show.  The step, the neutral
fractions and kappa must be identical (same kernels, FP64)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import hii as H  # noqa: E402
from synth import workloads as W  # noqa: E402


def _sw():
    import paper_2207_12848_amd as sw
    return sw


def _call(sw, fn, dag, ab, y, p):
    prm = sw._binding.sweep_ion_params_t()
    for k in ("n_H", "sigma_H", "alpha_B", "photon_rate", "length_unit", "dt_max", "courant"):
        setattr(prm, k, float(p[k]))
    C = dag.n_cells
    yg = torch.tensor(y, device="cuda")
    kap = torch.full((C, 1), -1.0, dtype=torch.float32, device="cuda")
    a = torch.tensor(ab[:, None], device="cuda")
    dt = ctypes.c_double()
    sw._binding.check(fn(dag.handle, int(a.data_ptr()), ctypes.byref(prm), 1e30, int(yg.data_ptr()),
                         int(kap.data_ptr()), ctypes.byref(dt), None))
    torch.cuda.synchronize()
    return dt.value, yg.cpu().numpy(), kap.cpu().numpy()


def test_noalloc_ion_step_matches_allocating_step():
    sw = _sw()
    rng = np.random.default_rng(11)
    out = []
    for n, scale in ((16, 1.0), (8, 1e-3)):  # the second mesh is smaller, its limit larger
        w = W.hii_rtype(n, 8)
        p = dict(w["hii"])
        p["dt_max"] = 1e30  # the limit decides the step
        dag = sw.build_dag(w["meshes"], w["dirs"])
        C = n ** 3
        y = rng.uniform(0.05, 1.0, C)
        ab = (scale * rng.uniform(0.0, 1e-3, C)).astype(np.float32)
        ref = _call(sw, sw._binding.sweep_ion_step, dag, ab, y, p)
        got = _call(sw, sw._binding.sweep_ion_step_noalloc, dag, ab, y, p)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
        V = w["meshes"][0]["cell_volume"] * p["length_unit"] ** 3
        lim = p["courant"] * H.ion_limit(ab.astype(np.float64), y, V, p)
        assert abs(got[0] - lim) <= 1e-12 * lim
        out.append(got[0])
        dag.close()
    assert out[1] > out[0]
