"""Host-side checks: the seeded scene generators and the benchmark CLI guard."""
import json
import os
import subprocess
import sys

import numpy as np

from paper_2402_01181_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_env(env):
    assert env.x.dtype == np.float32 and env.x.shape == (env.N, 3)
    assert env.C.shape == (env.N, 3, 3) and env.F.shape == (env.N, 3, 3)
    for k in ("E", "nu", "rho", "V0"):
        v = getattr(env, k)
        assert v == float(np.float32(v))          # FP32-representable scalars
    dx = 1.0 / env.n
    # every particle's stencil sits inside the grid and above the boundary band
    base = np.floor(env.x.astype(np.float64) * env.n - 0.5)
    assert base.min() >= 2 and base.max() <= env.n - 4


def test_scene_sizes_and_determinism():
    c = scenes.cube_scene()
    assert c.envs[0].N == 8192 and c.envs[0].n == 32 and c.dt == float(np.float32(1e-4))
    s = scenes.slab_scene(substeps=10)
    assert s.envs[0].N == 30000 and s.envs[0].n == 64 and len(s.envs[0].tools) == 1
    assert np.array_equal(s.envs[0].x, scenes.slab_scene(substeps=10).envs[0].x)   # seeded
    assert not np.array_equal(s.envs[0].x, scenes.slab_scene(seed=3, substeps=10).envs[0].x)
    for sc in (c, s):
        for env in sc.envs:
            _check_env(env)
    d = scenes.diff_scene()
    assert d.envs[0].tools[0].traj.shape == (200, 3) and d.extra["checkpoint_every"] == 20
    b = scenes.batched_scene(n_envs=12)
    assert len(b.envs) == 12 and all(5000 <= e.N <= 50000 and e.n in (32, 64) for e in b.envs)
    assert all(3e3 <= e.E <= 3e4 and 0.25 <= e.nu <= 0.45 for e in b.envs)
    for env in b.envs:
        _check_env(env)


def test_large_scene_shape():
    sc = scenes.large_slab_scene(substeps=500)
    env = sc.envs[0]
    assert env.N == 1 << 20 and env.n == 128
    assert env.tools[0].traj.shape == (500, 3) and env.tools[0].contact == scenes.CONTACT_STICKY
    speeds = np.linalg.norm(env.tools[0].traj.astype(np.float64), axis=1)
    np.testing.assert_allclose(speeds, 0.2, rtol=1e-6)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_shipped_tuning_table_is_well_formed():
    """The launch-shape table shipped for the benchmark workloads holds
    options the library accepts."""
    import json
    from paper_2402_01181_amd import _lib as L
    from paper_2402_01181_amd.autotune import SHIPPED, shipped
    table = json.load(open(SHIPPED))
    assert table
    for key, entry in table.items():
        opts = shipped(key)
        assert opts == {int(k): int(v) for k, v in entry["options"].items()}
        assert opts[L.OPT_SCHEME] == L.SCHEME_TILED
        assert opts[L.OPT_BLOCK] in (64, 128, 256)
        assert 16 <= opts[L.OPT_ITEM] <= 4096 and opts[L.OPT_ITEM] % 16 == 0
        assert opts[L.OPT_SORT_EVERY] >= 1 and opts[L.OPT_NODE_SLOTS] in (1, 3)
    assert shipped("no such workload") is None
