"""The binding rejects mis-sized, mistyped or host arrays before any call
reaches the library (CPU only: every case raises before a kernel launch)."""
import pytest
import torch

from paper_2202_02840_amd import _lib
from paper_2202_02840_amd._lib import HNET_PARAMS, Context


@pytest.fixture(autouse=True)
def host_as_device(monkeypatch):
    # host tensors stand in for device tensors, so that each case reaches
    # the check it is about (every case still raises before a library call)
    monkeypatch.setattr(_lib, "_on_device", lambda t: True)


def ctx_stub(n):
    # a Context without a device handle: every checked method must raise
    # before it touches the library
    c = object.__new__(Context)
    c._h = None
    c.n = n
    c.device = torch.device("cpu")
    return c


def f64(*shape):
    return torch.zeros(*shape, dtype=torch.float64)


def f32(*shape):
    return torch.zeros(*shape, dtype=torch.float32)


def corr(n):
    return dict(A=f64(n), B=f64(3, n), gA=f64(3, n), gB=f64(9, n))


def test_network_size():
    assert HNET_PARAMS == 4801


@pytest.mark.parametrize("case", ["short_v", "v_rows", "m_len", "gB_rows", "rho_len", "dtype"])
def test_derivatives_shapes(case):
    n = 10
    c = ctx_stub(n)
    args = dict(v=f64(3, n), m=f64(n), u=f64(n), rho=None, V=f64(n), corr=corr(n))
    if case == "short_v":
        args["v"] = f64(3, n - 1)
    elif case == "v_rows":
        args["v"] = f64(2, n)
    elif case == "m_len":
        args["m"] = f64(n + 1)
    elif case == "gB_rows":
        args["corr"]["gB"] = f64(6, n)
    elif case == "rho_len":
        args["rho"] = f64(n - 2)
    elif case == "dtype":
        args["u"] = f32(n)
    err = TypeError if case == "dtype" else ValueError
    with pytest.raises(err, match="expected"):
        c.derivatives(None, **args)


def test_host_tensor_refused(monkeypatch):
    monkeypatch.setattr(_lib, "_on_device", lambda t: t.is_cuda)
    n = 6
    c = ctx_stub(n)
    with pytest.raises(ValueError, match="device tensors"):
        c.derivatives(None, f64(3, n), f64(n), f64(n), None, f64(n), corr(n))


def test_component_layouts_accepted():
    # [k, n] and flat [k n] both pass; [n, k] does not
    n = 4
    for v in (f64(3, n), f64(3 * n)):
        _lib._arr(v, "v", 3, n)
    with pytest.raises(ValueError, match="expected shape"):
        _lib._arr(f64(n, 3), "v", 3, n)
    with pytest.raises(ValueError, match="contiguous"):
        _lib._arr(f64(n, 3).t(), "v", 3, n)


def test_corrections_and_moments_shapes():
    n = 8
    c = ctx_stub(n)
    mom = dict(m0=f64(n), m1=f64(3, n), m2=f64(6, n), gm0=f64(3, n), gm1=f64(9, n), gm2=f64(17, n))
    with pytest.raises(ValueError, match="gm2"):
        c.corrections(mom)


def test_compatible_energy_shapes():
    n = 5
    c = ctx_stub(n)
    with pytest.raises(ValueError, match="pk"):
        c.compatible_energy(None, f64(3, n), f64(n), f64(n), None, f64(n), corr(n), f64(9, n),
                            f64(3, n), 1e-3, pk=f64(3, n + 1))
    with pytest.raises(ValueError, match="dpdt"):
        c.compatible_energy(None, f64(3, n), f64(n), f64(n), None, f64(n), corr(n), f64(9, n),
                            f64(n), 1e-3)


def test_per_particle_calls():
    n = 7
    c = ctx_stub(n)
    with pytest.raises(ValueError, match="H_sorted"):
        c.hsolve(64.0, f64(n + 1))
    with pytest.raises(ValueError, match="H_sorted"):
        c.update_support(f64(n - 1))
    with pytest.raises(ValueError, match="H_sorted"):
        c.hnet_features(64.0, f64(2 * n))
    with pytest.raises(ValueError, match="src"):
        c.permute(f64(3, n + 1), True)
    with pytest.raises(ValueError, match="gradv"):
        c.timestep(None, f64(n), f64(n), None, f64(n), f64(3, n))
    with pytest.raises(ValueError, match="dpdt"):
        c.time_levels(None, f64(n), f64(n), 0.1, 0.1)


def test_build_shapes():
    c = ctx_stub(0)
    with pytest.raises(ValueError, match="H"):
        c.build_cells(f64(9), f64(9), f64(9), f64(8), None)
    with pytest.raises(ValueError, match="x"):
        c.build_cells(f64(3, 3), f64(9), f64(9), f64(9), None)
    with pytest.raises(ValueError, match="box_offsets"):
        c.build_cells_batch([0], f64(9), f64(9), f64(9), f64(9), None)


def test_step_and_verlet_io():
    n = 6
    c = ctx_stub(0)
    dev = dict(x=f64(n), y=f64(n), z=f64(n), H=f64(n), v=f64(3, n), m=f64(n), u=f64(n), rho=None)
    io = dict(dev)
    io.update(perm=torch.zeros(n, dtype=torch.int32), V=f64(n), m0=f64(n), m1=f64(3, n),
              m2=f64(6, n), gm0=f64(3, n), gm1=f64(9, n), gm2=f64(18, n), A=f64(n), B=f64(3, n),
              gA=f64(3, n), gB=f64(9, n), gradv=f64(9, n), dpdt=f64(3, n), dudt=f64(n))
    bad = dict(io, gm1=f64(9, n - 1))
    with pytest.raises(ValueError, match="gm1"):
        c._io(bad)
    bad = dict(io, perm=f64(n))
    with pytest.raises(TypeError, match="perm"):
        c._io(bad)
    st = dict(dev, dpdt=f64(3, n), dudt=f64(n + 1))
    with pytest.raises(ValueError, match="dudt"):
        c.verlet_step(st, None, 1e-3)


def test_network_calls():
    c = ctx_stub(0)
    nb = 16
    theta, m, v = f32(HNET_PARAMS), f32(HNET_PARAMS), f32(HNET_PARAMS)
    with pytest.raises(ValueError, match="theta"):
        c.hnet_forward(f32(HNET_PARAMS - 1), f32(8, nb))
    with pytest.raises(ValueError, match="feat"):
        c.hnet_forward(theta, f32(7, nb))
    with pytest.raises(TypeError, match="feat"):
        c.hnet_forward(theta, f64(8, nb))
    with pytest.raises(ValueError, match="target"):
        c.hnet_train_step(theta, m, v, 1, 1e-3, f32(8, nb), f32(nb + 1))
    with pytest.raises(ValueError, match="^m:"):
        c.hnet_train_step(theta, f32(10), v, 1, 1e-3, f32(8, nb), f32(nb))
    with pytest.raises(ValueError, match="grad"):
        c.hnet_train_step_noalloc(theta, m, v, 1, 1e-3, f32(8, nb), f32(nb), grad=f32(5))
    with pytest.raises(ValueError, match="H_conv"):
        c.hnet_targets(f64(nb), f64(nb - 1))
    c.n = 9
    with pytest.raises(ValueError, match="H_prev_sorted"):
        c.hnet_seed(theta, 64.0, f64(8))
