"""The Python binding checks every device buffer before it hands a pointer to the C ABI
(which sees no sizes): wrong type, dtype, shape, contiguity or device raise a Python
error and nothing is launched.  Runs on the CPU: the checks fire before any HIP call, so
an operator object without a built handle stands in for a real one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
wf = pytest.importorskip("paper_2605_26347_amd")


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"{name} reached the C ABI")


def fake_operator(nchan=2, nx=8, ny=6, rows=10):
    op = object.__new__(wf.Operator)
    op._lib = _NoLib()
    op._h = None
    op.nchan, op.nx, op.ny, op.nrows_total, op.device = nchan, nx, ny, rows, 0
    return op


def img(op, dtype=torch.float32):
    return torch.zeros((op.nchan, op.ny, op.nx), dtype=dtype)


def test_rejects_non_tensor():
    op = fake_operator()
    with pytest.raises(TypeError, match="torch.Tensor"):
        op.psf_apply(np.zeros((2, 6, 8), np.float32), out=img(op, torch.complex64))


@pytest.mark.parametrize("call", ["forward", "psf_apply", "psf_apply_re", "layer_grid"])
def test_rejects_wrong_input_dtype(call):
    op = fake_operator()
    x = img(op, torch.float64)
    with pytest.raises(TypeError, match="dtype"):
        if call == "layer_grid":
            op.layer_grid(0, 0, x, out=torch.zeros((12, 16), dtype=torch.complex64))
        else:
            getattr(op, call)(x, out=torch.zeros(1))


def test_rejects_wrong_shape_and_undersized_output():
    op = fake_operator()
    with pytest.raises(ValueError, match="shape"):
        op.psf_apply(torch.zeros((2, 6, 7)), out=img(op, torch.complex64))
    with pytest.raises(ValueError, match="shape"):
        op.forward(img(op), out=torch.zeros(9, dtype=torch.complex64))
    with pytest.raises(ValueError, match="shape"):
        op.adjoint(torch.zeros(11, dtype=torch.complex64), out=img(op, torch.complex64))


def test_rejects_non_contiguous():
    op = fake_operator(nchan=1, nx=6, ny=6)
    x = torch.zeros((1, 6, 6)).transpose(1, 2)
    assert x.shape == (1, 6, 6) and not x.is_contiguous()
    with pytest.raises(ValueError, match="contiguous"):
        op.psf_apply_re(x, out=torch.zeros((1, 6, 6)))


def test_rejects_host_tensor():
    op = fake_operator()
    with pytest.raises(ValueError, match="cuda"):
        op.psf_apply(img(op), out=img(op, torch.complex64))
    with pytest.raises(ValueError, match="cuda"):
        op.dirty_image(torch.zeros(10, dtype=torch.complex64), out=img(op))
    with pytest.raises(ValueError, match="cuda"):
        op.fb_iterate(img(op), img(op), 1, 0.5, 0.0)


def test_rejects_wrong_graph_and_autotune_buffers():
    op = fake_operator()
    with pytest.raises(ValueError, match="shape"):
        op.capture("adjoint", torch.zeros(9, dtype=torch.complex64), img(op, torch.complex64),
                   None)
    with pytest.raises(TypeError, match="dtype"):
        op.autotune(img(op), img(op, torch.complex64))


def test_network_checks():
    net = object.__new__(wf.Network)
    net._lib = _NoLib()
    net._h = None
    with pytest.raises(ValueError, match="shape"):
        net.infer(torch.zeros((4, 4)))
    with pytest.raises(TypeError, match="dtype"):
        net.loss_grad(torch.zeros((4, 5)), torch.zeros((4, 450), dtype=torch.float64))
    with pytest.raises(ValueError, match="cuda"):
        net.train(torch.zeros((4, 5)), torch.zeros((4, 450)))
    with pytest.raises(TypeError, match="dtype"):
        wf.Network.targets(torch.zeros(3, dtype=torch.float32), torch.zeros(3))
