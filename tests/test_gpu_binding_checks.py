"""The binding refuses device arrays the library would read or write out of
bounds (too short, wrong dtype, not contiguous) and host arrays that are too
short, before anything reaches the library: each case is one entry point
with one bad argument and otherwise valid inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    c = Context(0, 1 << 30)
    yield c
    c.close()


def _f64(*shape):
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def _f32(*shape):
    return torch.zeros(shape, dtype=torch.float32, device="cuda")


def _i32(*shape):
    return torch.zeros(shape, dtype=torch.int32, device="cuda")


def test_short_or_mistyped_arrays_are_refused(ctx):
    from paper_1502_07873_amd import EigError, make_prior
    from paper_1502_07873_amd.query import device_medium
    _say("binding argument checks")
    prior = make_prior(-np.ones(7), np.ones(7))
    n = 3
    H = _f64(n, 7, 7)
    w = np.full(n, 1.0 / n)
    # laplace_eig
    with pytest.raises(EigError, match="dkl"):
        ctx.laplace_eig(H, prior, w, _f64(n - 1), _f64(1))
    with pytest.raises(EigError, match="eig"):
        ctx.laplace_eig(H, prior, w, _f64(n), _f32(1))
    with pytest.raises(EigError, match="status"):
        ctx.laplace_eig(H, prior, w, _f64(n), _f64(1), status=_f64(n))
    with pytest.raises(EigError, match="w: expected at least"):
        ctx.laplace_eig(H, prior, w[:2], _f64(n), _f64(1))
    with pytest.raises(EigError, match="H1"):
        ctx.laplace_eig(_f64(n, 7, 7).transpose(1, 2), prior, w, _f64(n), _f64(1))
    # design_eval / design_greedy
    C = 4
    Hr = _f64(n, C, 7, 7)
    with pytest.raises(EigError, match="mask"):
        ctx.design_eval(Hr, _i32(2, C), prior, w, _f64(2))
    with pytest.raises(EigError, match="eig"):
        ctx.design_eval(Hr, torch.ones((2, C), dtype=torch.uint8, device="cuda"), prior, w,
                        _f64(1))
    with pytest.raises(EigError, match="order"):
        ctx.design_greedy(Hr, prior, w, 3, _i32(2), _f64(3))
    with pytest.raises(EigError, match="curve"):
        ctx.design_greedy(Hr, prior, w, 3, _i32(3), _f64(2))
    # nested_mc_eig
    g = _f32(5, 6)
    with pytest.raises(EigError, match="logratio"):
        ctx.nested_mc_eig(g, g, g, 0.1, _f64(4))
    with pytest.raises(EigError, match="g_inner"):
        ctx.nested_mc_eig(g, g, torch.zeros((5, 6), dtype=torch.float64, device="cuda"), 0.1,
                          _f64(5))
    # solves: traces / nominal / J / H1 / noise sized from grid and receivers
    grid = (40, 30, 10.0, 1e-3, 10, 0)
    med = device_medium("layered", np.full(30, 2500.0), np.full(30, 2e10), np.full(30, 1e10))
    rec = np.array([3, 9, 20], dtype=np.int32)
    th = np.array([200.0, 150.0, 0.02, 20.0, 1e14, 1e14, 1e14])
    with pytest.raises(EigError, match=r"traces\[0\]"):
        ctx.forward_solve_batch([grid], [med], th, [rec], [_f32(11, 3, 1)])
    with pytest.raises(EigError, match="H1"):
        ctx.jacobian_fd([grid], [med], th, [rec], 1.0, _f64(1, 7, 7), per_receiver=True)
    with pytest.raises(EigError, match=r"nominal\[0\]"):
        ctx.jacobian_fd([grid], [med], th, [rec], 1.0, _f64(1, 7, 7), nominal=[_f32(10, 3, 2)])
    with pytest.raises(EigError, match=r"J\[0\]"):
        ctx.jacobian_sensitivity([grid], [med], th, [rec], 1.0, _f64(1, 7, 7),
                                 J=[_f64(11, 3, 2, 6)])
    with pytest.raises(EigError, match="theta"):
        ctx.jacobian_fd([grid], [med], th[:6], [rec], 1.0, _f64(1, 7, 7))
    with pytest.raises(EigError, match=r"noise\[0\]"):
        ctx.theorem3_eig([grid], [med], th, [rec], [_f32(11, 3)], 0.1, prior, [1.0],
                         _f64(1, 7, 7), _f64(1, 7, 7), _f64(1))
    with pytest.raises(EigError, match="H2"):
        ctx.theorem3_eig([grid], [med], th, [rec], [_f32(11, 3, 2)], 0.1, prior, [1.0],
                         _f64(1, 7, 7), _f64(1, 7, 6), _f64(1))
    torch.cuda.synchronize()
