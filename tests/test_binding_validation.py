"""CPU checks of the Python binding's argument validation: shapes, sizes and
dtypes are checked before any call into the library, so a wrong buffer is a
ValueError and never an out-of-bounds read or write."""
import numpy as np
import pytest

from paper_1702_02207_amd import osc


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import os
    if not os.path.exists(osc.LIB_PATH):
        pytest.skip("libosc.so not built")
    osc.load()


def _chain(batch=3, s=4):
    return np.ones((batch, s)), np.full((batch, s), 100.0)


def test_chain_scalar_dt_is_broadcast():
    m, k = _chain()
    sysm = osc.System("chain", "rk4", "f32", m, k, 1e-3)
    assert sysm.batch == 3 and sysm.s == 4
    assert sysm._keep[2].shape == (3,) and np.all(sysm._keep[2] == 1e-3)


@pytest.mark.parametrize("dt", [np.ones(2) * 1e-3, np.ones(4) * 1e-3])
def test_chain_dt_of_wrong_length_rejected(dt):
    m, k = _chain()
    with pytest.raises(ValueError, match="dt"):
        osc.System("chain", "rk4", "f32", m, k, dt)


def test_chain_k_shape_must_match_m():
    m, k = _chain()
    with pytest.raises(ValueError, match="chain M and K"):
        osc.System("chain", "rk4", "f32", m, k[:, :3], 1e-3)
    with pytest.raises(ValueError, match="chain M and K"):
        osc.System("chain", "rk4", "f32", m[0], k[0], 1e-3)


def test_chain_batch_argument_must_agree():
    m, k = _chain()
    with pytest.raises(ValueError, match="disagrees"):
        osc.System("chain", "rk4", "f32", m, k, 1e-3, batch=5)


def test_dense_shapes_checked():
    M = np.eye(5)
    with pytest.raises(ValueError, match="shared dense"):
        osc.System("dense", "rk4", "f32", M, np.eye(4), [1e-2], shared=True, batch=2)
    with pytest.raises(ValueError, match="shared dense"):
        osc.System("dense", "rk4", "f32", np.ones((5, 4)), np.ones((5, 4)), [1e-2], shared=True, batch=2)
    with pytest.raises(ValueError, match="batch must be given"):
        osc.System("dense", "rk4", "f32", M, M, [1e-2], shared=True)
    with pytest.raises(ValueError, match="per-instance dense"):
        osc.System("dense", "rk4", "f32", M, M, [1e-2], shared=False)
    with pytest.raises(ValueError, match="dt must hold"):
        osc.System("dense", "rk4", "f32", np.stack([M] * 3), np.stack([M] * 3), [1e-2, 1e-2], shared=False)
    sysm = osc.System("dense", "rk4", "f32", np.stack([M] * 3), np.stack([M] * 3), 1e-2, shared=False)
    assert sysm.batch == 3 and sysm._keep[2].shape == (3,)


def test_unknown_enums_rejected():
    m, k = _chain()
    with pytest.raises(ValueError, match="unknown"):
        osc.System("chain", "rk5", "f32", m, k, 1e-3)
    with pytest.raises(ValueError, match="unknown"):
        osc.System("ring", "rk4", "f32", m, k, 1e-3)


def test_state_checked_before_any_call():
    import torch
    m, k = _chain()
    sysm = osc.System("chain", "rk4", "f32", m, k, 1e-3)
    x = torch.zeros(3, 4)
    with pytest.raises(ValueError, match="not been created"):
        sysm.integrate(x, x, 10)
    sysm.handle = object()          # stands in for a created handle; no call is made
    try:
        with pytest.raises(ValueError, match="CUDA tensor"):
            sysm.integrate(x, x, 10)
        with pytest.raises(ValueError, match="CUDA tensor"):
            sysm.energy(x, x)
    finally:
        sysm.handle = None


def test_server_submit_checks_sizes():
    with osc.Server(max_slots=4, fake_executor=True) as srv:
        x0 = np.zeros(4, dtype=np.float32)
        with pytest.raises(ValueError, match="needs 4 values"):
            srv.submit("chain", "rk4", "f32", np.ones(3), np.ones(4), [1e-3], x0, x0, 10)
        with pytest.raises(ValueError, match="needs 16 values"):
            srv.submit("dense", "rk4", "f32", np.eye(4), np.ones(4), [1e-3], x0, x0, 10)
        with pytest.raises(ValueError, match="same number of DOFs"):
            srv.submit("chain", "rk4", "f32", np.ones(4), np.ones(4), [1e-3], x0, x0[:3], 10)
        with pytest.raises(ValueError, match="one step size"):
            srv.submit("chain", "rk4", "f32", np.ones(4), np.ones(4), [1e-3, 1e-3], x0, x0, 10)
        t = srv.submit("chain", "rk4", "f32", np.ones(4), np.full(4, 10.0), [1e-3], x0, x0, 10)
        r = srv.wait(t, timeout=10.0)
        assert r["x_end"].shape == (4,)
