"""GPU parity of the proposal network's kernels (sfw_net_*) against the FP64 oracle.

The library computes with bf16 weights, inputs and activations (float32 accumulation). The
oracle is fed the same bf16-rounded weights and input, so what remains is the rounding of the
three hidden activations and of the backward gradients to bf16 (half an ulp = 2^-9 relative,
about 0.2 % RMS per rounding): relative L2 <= 2e-2 for the output and <= 5e-2 for the weight
gradients, which pass through up to three more roundings. Volumes have ragged tiles (18 and 75
half-resolution voxels along x against 64-voxel tiles, 6 and 10 along y against 4-row tiles),
odd sizes and a tiny 3 x 4 x 5 case.
"""
import numpy as np
import pytest

from oracle import cnn
from tests._common import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05473_amd import _lib
    return _lib


def say(*msg):
    print("[case]", *msg, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(a, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in params]).astype(np.float32)


def split(vec, like):
    out, o = [], 0
    for w, b in like:
        out.append((vec[o:o + w.size].reshape(w.shape), vec[o + w.size:o + w.size + b.size]))
        o += w.size + b.size
    return out


def params_and_input(seed, shape):
    rng = np.random.default_rng(seed)
    params = [(w, 0.1 * rng.standard_normal(b.shape)) for w, b in cnn.init_params(rng)]
    x = rng.standard_normal(shape).astype(np.float32)
    return rng, params, x


def oracle_params(params):
    return [(bf16(w), np.asarray(b, dtype=np.float32).astype(np.float64)) for w, b in params]


@pytest.mark.parametrize("shape", [(12, 20, 36), (7, 9, 33), (6, 12, 150), (3, 4, 5)])
def test_forward_parity(L, shape):
    rng, params, x = params_and_input(11, shape)
    scale = 0.7
    say("sfw_net_forward", shape)
    with L.Net(shape) as net:
        assert net.num_params == flat(params).size
        net.set_params(flat(params))
        out = net.forward(dev(x), scale)
        torch.cuda.synchronize()
        got = np.moveaxis(out.cpu().numpy()[..., :3], -1, 0)
    want, _ = cnn.forward(oracle_params(params), bf16(x * np.float32(scale))[None])
    assert got.shape == want.shape
    assert rel_l2(got, want) <= 2e-2
    for c in range(3):
        assert rel_l2(got[c], want[c]) <= 3e-2, c


@pytest.mark.parametrize("shape", [(12, 20, 36), (6, 12, 150)])
def test_gradients_parity(L, shape):
    rng, params, x = params_and_input(12, shape)
    scale = 0.5
    Z, Y, X = shape
    atoms = np.column_stack([rng.uniform(0.5, 2, 5), rng.uniform(1, X - 2, 5),
                             rng.uniform(1, Y - 2, 5), rng.uniform(0.5, Z - 1.5, 5),
                             rng.uniform(1, 2, 5), rng.uniform(1.5, 2.5, 5)])
    say("sfw_net_gradients", shape)
    with L.Net(shape) as net:
        net.set_params(flat(params))
        loss, grads = net.gradients(dev(x), scale, atoms)
    op = oracle_params(params)
    out, cache = cnn.forward(op, bf16(x * np.float32(scale))[None])
    lo, dout = cnn.loss(out, atoms.astype(np.float32).astype(np.float64))
    want = cnn.backward(op, cache, dout)
    assert abs(loss - lo) <= 3e-2 * lo
    got = split(grads, params)
    for layer in range(4):
        assert rel_l2(got[layer][0], want[layer][0]) <= 5e-2, ("w", layer)
        assert rel_l2(got[layer][1], want[layer][1]) <= 5e-2, ("b", layer)


def test_training_lowers_the_loss_and_propose_reads_the_maximum(L):
    shape = (16, 24, 32)
    rng, params, x = params_and_input(13, shape)
    atoms = np.array([[1.0, 10.0, 8.0, 6.0, 1.4, 2.0], [1.0, 22.0, 15.0, 9.0, 1.8, 1.7]])
    say("sfw_net_train_step x 40, sfw_net_propose", shape)
    with L.Net(shape) as net:
        net.set_params(flat([(w, np.zeros_like(b)) for w, b in params]))
        X = dev(x)
        first = net.train_step(X, 1.0, atoms, 1e-3, want_loss=True)
        for _ in range(38):
            net.train_step(X, 1.0, atoms, 1e-3)
        last = net.train_step(X, 1.0, atoms, 1e-3, want_loss=True)
        p = net.get_params()
        assert np.all(np.isfinite(p)) and not np.array_equal(p, flat(params))
        out = net.forward(X, 1.0).cpu().numpy()
        theta, score = net.propose(X, 1.0)
    assert last < 0.5 * first
    h = out[..., 0]
    o = np.unravel_index(np.argmax(h), h.shape)  # first maximum in C order
    assert score == pytest.approx(float(h[o]))

    def offset(axis):  # parabola through log max(h, 1e-3) at the maximum and its neighbours
        if o[axis] == 0 or o[axis] + 1 == h.shape[axis]:
            return 0.0
        lo, hi = list(o), list(o)
        lo[axis] -= 1
        hi[axis] += 1
        a, b, c = (np.log(max(float(h[tuple(i)]), 1e-3)) for i in (lo, o, hi))
        den = a - 2 * b + c
        return 0.0 if not den < 0 else float(np.clip(0.5 * (a - c) / den, -0.5, 0.5))

    want = [2.0 * (o[2] + offset(2)), 2.0 * (o[1] + offset(1)), 2.0 * (o[0] + offset(0))]
    assert np.allclose(theta[:3], want, atol=1e-5)
    assert theta[3] == pytest.approx(float(out[o][1])) and theta[4] == pytest.approx(float(out[o][2]))


def test_net_rejects_bad_inputs(L):
    say("sfw_net argument checks")
    with L.Net((8, 8, 8)) as net:
        with pytest.raises(L.SfwError):
            net.forward(dev(np.zeros((10, 8, 8))), 1.0)  # beyond vol_max
        x = dev(np.zeros((8, 8, 8)))
        with pytest.raises(L.SfwError):
            net.gradients(x, 1.0, np.zeros((97, 6)))  # more than 96 atoms
        with pytest.raises(L.SfwError):
            net.set_params(np.zeros(5))
        # the solver takes a proposal network only on its workspace's stream
        other = torch.cuda.Stream()
        with L.Workspace((8, 8, 8), (3, 3, 3), 8, stream=other) as ws:
            H = dev(np.full((3, 3, 3), 1.0 / 27))
            opts = L.default_options()
            opts.proposal = net.handle.value
            with pytest.raises(L.SfwError) as e:
                L.sfw_solve(ws, x, H, 1.0, opts)
            assert e.value.code == L.SFW_EINVAL and "stream" in str(e.value)
