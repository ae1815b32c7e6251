"""GPU parity of the differentiable form: the hand-written adjoint against
the FP64 oracle gradient, and the autograd wiring against central finite
differences of the GPU forward."""
import numpy as np
import pytest

from oracle import epic_oracle as O
from paper_1603_02126_amd import synth

pytestmark = pytest.mark.gpu


def _setup(wl, seed=1):
    import torch
    from paper_1603_02126_amd import lib
    a = wl.array
    packed = synth.make_efield(wl)
    plan = lib.Plan([a])
    dev = plan.device
    e = torch.from_numpy(packed).to(dev)
    rng = np.random.default_rng(seed)
    g = wl.g_true * (1 + 0.05 * (rng.standard_normal(wl.g_true.shape) + 1j * rng.standard_normal(wl.g_true.shape)))
    return plan, packed, e, g


def _oracle_grad(wl, packed, g, M, channels):
    a = wl.array
    cells = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    E = O.unpack(packed, a.efmt)
    out = []
    for c in channels:
        I = O.image_fixed_gains(E[:, c], g[c], cells, a.nx, a.ny, float(a.n_ant))
        out.append(O.image_gain_gradient(E[:, c], g[c], cells, a.nx, a.ny, float(a.n_ant), 2 * (I - M[c])))
    return np.array(out)


def _edge_layout(wl, seed=5):
    """Kernels that straddle columns 31/32 or wrap around the last column and
    row (the paired adjoint degrids each half of the columns separately)."""
    a = wl.array
    na = a.n_ant
    rng = np.random.default_rng(seed)
    k = na // 3
    px = np.concatenate([rng.uniform(31.0, 32.0, k), rng.uniform(63.0, 64.0, k), rng.uniform(5.0, 58.0, na - 2 * k)])
    py = np.concatenate([rng.uniform(3.0, 60.0, 2 * k), rng.uniform(63.0, 64.0, na - 2 * k)])
    xy = np.column_stack([a.x0 + px * a.dx, a.y0 + py * a.dy])
    return wl.replace(array=synth.dataclasses.replace(a, ant_xy=xy))


@pytest.mark.parametrize("n,na,efmt,kernel,edges", [(32, 48, synth.FMT_CI8, 2, False), (64, 200, synth.FMT_CI4, 2, False),
                                                     (16, 30, synth.FMT_CF32, 1, False),
                                                     (64, 180, synth.FMT_CI8, 1, False),
                                                     (64, 150, synth.FMT_CI4, 2, True)])
def test_adjoint_matches_oracle_gradient(cuda, n, na, efmt, kernel, edges):
    import torch
    from paper_1603_02126_amd.autograd import epic_image
    wl = synth.config_small(n=n, n_ant=na, efmt=efmt, kernel=kernel, n_chan=2, n_samples=53)
    if edges:
        wl = _edge_layout(wl)
    plan, packed, e, g = _setup(wl)
    M = np.random.default_rng(3).uniform(0, 1, size=(2, n, n)) * 0.5
    gt = torch.from_numpy(g.astype(np.complex64)).to(cuda).requires_grad_(True)
    img = epic_image(gt, plan, 0, e, wl.n_samples)
    loss = ((img.double() - torch.from_numpy(M).to(cuda)) ** 2).sum()
    loss.backward()
    got = gt.grad.cpu().numpy().astype(np.complex128)
    ref = _oracle_grad(wl, packed, g.astype(np.complex64).astype(np.complex128), M, [0, 1])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= 1e-4, err
    plan.close()


def test_autograd_central_differences(cuda):
    """16 random gains, h = 1e-3, central differences of the GPU forward."""
    import torch
    from paper_1603_02126_amd.autograd import epic_image
    wl = synth.config_small(n=32, n_ant=48, n_chan=1, n_samples=40)
    plan, packed, e, g = _setup(wl, seed=9)
    M = np.random.default_rng(4).uniform(0, 1, size=(1, 32, 32)) * 0.5
    Mt = torch.from_numpy(M).to(cuda)

    def loss_of(gg):
        img = epic_image(gg, plan, 0, e, wl.n_samples)
        return ((img.double() - Mt) ** 2).sum()

    g0 = torch.from_numpy(g).to(cuda)
    gl = g0.clone().requires_grad_(True)
    loss_of(gl).backward()
    grad = gl.grad.cpu().numpy()
    h = 1e-3
    idx = np.random.default_rng(2).choice(wl.array.n_ant, 16, replace=False)
    fd = []
    for a in idx:
        d = torch.zeros_like(g0)
        d[0, a] = h
        dre = (loss_of(g0 + d) - loss_of(g0 - d)).item() / (2 * h)
        dim = (loss_of(g0 + 1j * d) - loss_of(g0 - 1j * d)).item() / (2 * h)
        fd.append(dre + 1j * dim)
    fd = np.array(fd)
    err = np.abs(grad[0, idx] - fd).max() / np.abs(fd).max()
    assert err <= 2e-3, err
    plan.close()


def model_image_gpu(wl, dev):
    """The loss target of the differentiable workload: the expected image of
    its 50 brightest model sources plus the receiver noise (data units), made
    by the library's fixed-gain imaging of a tone sky whose time average is
    that expectation exactly (unit gains, complex float samples)."""
    import torch
    from paper_1603_02126_amd import lib
    a = wl.array
    src, sigma = synth.loss_target_sky(wl)
    tones = synth.tone_efield(a.ant_xy, a.freq_hz, src, sigma)
    spec = synth.dataclasses.replace(a, efmt=synth.FMT_CF32)
    with lib.Plan([spec]) as plan:
        ones = torch.ones((a.n_chan, a.n_ant), dtype=torch.complex128, device=dev)
        M = plan.image(0, torch.from_numpy(tones).to(dev), tones.shape[0], ones)
    return M, src, sigma


def test_adjoint_full_size_sampled_channels(cuda):
    """Differentiable workload at full size (256 antennas, 8+8-bit, 64
    channels, 64x64, 1000 samples), loss L = sum (I - M)^2 with M the model
    image of 50 point sources and the noise floor; the oracle checks M and the
    gradient on two channels."""
    import torch
    from paper_1603_02126_amd.autograd import epic_image
    wl = synth.config_diff()
    a = wl.array
    packed = synth.make_efield(wl, threads=8)
    from paper_1603_02126_amd import lib
    plan = lib.Plan([a])
    e = torch.from_numpy(packed).to(cuda)
    g = wl.g0
    Mt, src, sigma = model_image_gpu(wl, cuda)
    M = Mt.double().cpu().numpy()
    cells = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    for c in (0, 41):
        ref_M = O.model_image(cells, a.nx, a.ny, float(a.n_ant), a.ant_xy, a.freq_hz[c], src, sigma)
        assert np.abs(M[c] - ref_M).max() <= 1e-5 * np.abs(ref_M).max()
    gt = torch.from_numpy(g).to(cuda).requires_grad_(True)
    img = epic_image(gt, plan, 0, e, wl.n_samples)
    loss = ((img.double() - torch.from_numpy(M).to(cuda)) ** 2).sum()
    loss.backward()
    got = gt.grad.cpu().numpy()
    chans = [0, 41]
    ref = _oracle_grad(wl, packed[:, chans], g[chans], M[chans], [0, 1])
    err = np.abs(got[chans] - ref).max() / np.abs(ref).max()
    assert err <= 1e-4, err
    plan.close()
