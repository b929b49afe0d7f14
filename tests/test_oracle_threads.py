"""The threaded oracle run (orc_run_threads, used to time the oracle on the
host's cores) against the plain serial run: same substeps, same state.

Each node receives its P2G terms in particle order in both, so the results
must agree to the last bit; the test holds them to 1e-12 relative (the bound
the serial/threaded comparison is specified with) and reports the maximum
difference."""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes


def _run(orc, sc, S, threads):
    o = orc.Sim(sc.envs[0], sc.dt, gravity=sc.gravity, bound=sc.bound)
    o.run(S, threads=threads)
    return o


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("threads", [2, 3, 8, 64])
def test_threads_equal_serial_slab_with_tool(orc, threads):
    sc = scenes.small_slab_scene(seed=23, n_particles=3000, n=32, substeps=12, u=(0.05, -0.5, 0.0))
    sc.envs[0].tools[0].T0 = (sc.envs[0].tools[0].T0 - np.array([0, 0.012, 0])).astype(np.float32)
    a = _run(orc, sc, 12, None)
    b = _run(orc, sc, 12, threads)
    for f in ("x", "v", "C", "F"):
        r = _rel(getattr(b.state, f), getattr(a.state, f))
        assert r <= 1e-12, (f, r)
    np.testing.assert_array_equal(a.T, b.T)
    assert a.flags == b.flags


def test_threads_equal_serial_edge_cases(orc):
    """A frozen particle (stencil outside the grid), an inverted F and more
    threads than grid planes."""
    sc = scenes.small_slab_scene(seed=3, n_particles=400, n=8, substeps=4)
    env = sc.envs[0]
    env.x[0] = [0.01, 0.5, 0.5]
    env.F[1] = np.diag([1.0, 1.0, -0.5]).astype(np.float32)
    a = _run(orc, sc, 4, None)
    b = _run(orc, sc, 4, 16)
    for f in ("x", "v", "C", "F"):
        assert _rel(getattr(b.state, f), getattr(a.state, f)) <= 1e-12, f
    assert a.flags == b.flags
    assert a.flags & orc.FLAG_OUT_OF_DOMAIN and a.flags & orc.FLAG_INVERTED


def test_threads_equal_serial_cube(orc):
    sc = scenes.cube_scene(seed=1, substeps=10)
    a = _run(orc, sc, 10, None)
    b = _run(orc, sc, 10, 5)
    for f in ("x", "v", "C", "F"):
        assert np.array_equal(getattr(b.state, f), getattr(a.state, f)), f
