"""GPU parity of the learned path corrector (FP32 forward, backward, Adam and
the learned GNEB initial path) against the FP64 oracle network.

Tolerances (FP32 convolutions vs FP64): corrected images 1e-5 absolute per
component; loss 1e-5 relative; gradients max|g - g_ref| <= 1e-5 max|g_ref|
(weight-gradient sums accumulated in FP64; the FP32 activations and
back-propagated fields carry about 1e-7 relative error each); Adam 1e-6
relative.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import require_gpu, to_dev
from workloads import random_sphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def init_params(seed, scale=1.0):
    """He-style random parameters for the 10-16-16-16-3 network (float32)."""
    rng = np.random.default_rng(seed)
    ch = oracle.NET_CHANNELS
    out = []
    for l in range(4):
        fan = ch[l] * 27
        out.append(rng.standard_normal(ch[l + 1] * ch[l] * 27) * scale * np.sqrt(2.0 / fan))
        out.append(rng.standard_normal(ch[l + 1]) * 0.05)
    return np.concatenate(out).astype(np.float32)


def batch_case(L, B, seed):
    P = L[0] * L[1] * L[2]
    Sg = np.stack([random_sphere(P, seed + 3 * b) for b in range(B)])
    SA = np.stack([random_sphere(P, seed + 3 * b + 1) for b in range(B)])
    SB = np.stack([random_sphere(P, seed + 3 * b + 2) for b in range(B)])
    Ss = np.stack([random_sphere(P, seed + 100 + b) for b in range(B)])
    t = (np.arange(B, dtype=np.float32) + 1) / (B + 1)
    return Sg, SA, SB, Ss, t


def oracle_x(Sg, SA, SB, t):
    P = Sg.shape[-1]
    return np.concatenate([Sg, SA, SB, np.full((1, P), float(t))])


@pytest.mark.parametrize("L,scale", [((9, 7, 5), 1.0), ((16, 8, 4), 1.0), ((9, 7, 5), 2.0)])
def test_net_forward_matches_oracle(L, scale):
    # FP32 convolutions: the corrected image differs from the FP64 oracle by
    # about 1e-7 of the network output |u| per layer; the bound is 1e-5 for
    # He-scaled weights (|u| ~ 1) and 1e-5 * max|u| beyond that
    import torch
    from paper_2605_26016_amd import spx
    B = 3
    p32 = init_params(1, scale=scale)
    Sg, SA, SB, Ss, t = batch_case(L, B, 10)
    net = spx.Net()
    out = torch.zeros((B, 3, Sg.shape[-1]), dtype=torch.float64, device="cuda")
    spx.net_forward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), out)
    got = out.cpu().numpy()
    p64 = p32.astype(np.float64)
    for b in range(B):
        raw = oracle.net_forward(L, p64, oracle_x(Sg[b], SA[b], SB[b], t[b]))
        ref, _ = oracle.net_predict_loss(raw, Sg[b])
        tol = 1e-5 * max(1.0, float(np.max(np.abs(raw))))
        assert np.max(np.abs(got[b] - ref)) < tol, (b, np.max(np.abs(got[b] - ref)), tol)


def test_net_backward_matches_oracle():
    import torch
    from paper_2605_26016_amd import spx
    L = (7, 6, 5)
    B = 2
    p32 = init_params(2, scale=2.0)
    Sg, SA, SB, Ss, t = batch_case(L, B, 20)
    net = spx.Net()
    n = spx.net_nparams()
    assert n == oracle.net_nparams()
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    spx.net_backward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), to_dev(Ss), grad, loss)
    g = grad.cpu().numpy().astype(np.float64)
    p64 = p32.astype(np.float64)
    ref = np.zeros(n)
    lref = 0.0
    for b in range(B):
        lb, gb = oracle.net_backward(L, p64, oracle_x(Sg[b], SA[b], SB[b], t[b]), Sg[b], Ss[b])
        ref += gb / B
        lref += lb / B
    assert abs(loss.item() - lref) <= 1e-5 * lref
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    print(f"gradient max-normalised error {err:.2e}", flush=True)
    assert err <= 1e-5, err
    # deterministic
    grad2 = torch.zeros_like(grad)
    spx.net_backward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), to_dev(Ss), grad2)
    assert torch.equal(grad, grad2)


@pytest.mark.parametrize("L,dil", [((19, 13, 11), (1, 2, 4, 3)), ((12, 20, 9), (8, 4, 2, 1))],
                         ids=["d1243", "d8421"])
def test_net_dilated_forward_matches_oracle(L, dil):
    # dilated layers run as 3^3 tiles over the phase sub-grids of ceil(L/d)
    # sites: extents that are not multiples of d, sub-grids smaller than one
    # 8 x 8 x 4 tile, and a dilation of 8 on a 9-site axis (phases with one
    # and two sites)
    import torch
    from paper_2605_26016_amd import spx
    B = 2
    p32 = init_params(4, scale=1.5)
    Sg, SA, SB, _, t = batch_case(L, B, 40)
    P = L[0] * L[1] * L[2]
    net = spx.Net(dilation=dil)
    out = torch.zeros((B, 3, P), dtype=torch.float64, device="cuda")
    spx.net_forward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    p64 = p32.astype(np.float64)
    for b in range(B):
        raw = oracle.net_forward(L, p64, oracle_x(Sg[b], SA[b], SB[b], t[b]), dil=dil)
        ref, _ = oracle.net_predict_loss(raw, Sg[b])
        err = float(np.max(np.abs(got[b] - ref)))
        print(f"dilation {dil} image {b}: max |dS| {err:.2e}", flush=True)
        assert err <= 1e-5 * max(1.0, float(np.max(np.abs(raw)))), err
    # dilation 1 everywhere reproduces the undilated net
    spx.net_set_dilation(net, (1, 1, 1, 1))
    spx.net_forward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), out)
    raw = oracle.net_forward(L, p64, oracle_x(Sg[0], SA[0], SB[0], t[0]))
    ref, _ = oracle.net_predict_loss(raw, Sg[0])
    assert np.max(np.abs(out[0].cpu().numpy() - ref)) <= 1e-5 * max(1.0, float(np.max(np.abs(raw))))


def test_net_dilated_backward_matches_oracle():
    import torch
    from paper_2605_26016_amd import spx
    L = (11, 9, 7)
    B = 2
    dil = (2, 1, 3, 2)
    p32 = init_params(5, scale=2.0)
    Sg, SA, SB, Ss, t = batch_case(L, B, 50)
    net = spx.Net(dilation=dil)
    n = spx.net_nparams()
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    spx.net_backward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), to_dev(Ss), grad, loss)
    g = grad.cpu().numpy().astype(np.float64)
    p64 = p32.astype(np.float64)
    ref = np.zeros(n)
    lref = 0.0
    for b in range(B):
        lb, gb = oracle.net_backward(L, p64, oracle_x(Sg[b], SA[b], SB[b], t[b]), Sg[b], Ss[b], dil=dil)
        ref += gb / B
        lref += lb / B
    assert abs(loss.item() - lref) <= 1e-5 * lref
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    print(f"dilated gradient max-normalised error {err:.2e}", flush=True)
    assert err <= 1e-5, err


def test_net_dilation_is_validated():
    from paper_2605_26016_amd import spx
    net = spx.Net()
    for bad in ((0, 1, 1, 1), (1, 1, 65, 1)):
        with pytest.raises(spx.SpxError):
            spx.net_set_dilation(net, bad)


def test_mfma16_lane_layout_probe():
    # the 16x16x32 BF16 MFMA of the net's BF16 form, with the lane layout the
    # kernel assumes: small integers are exact in BF16 and their products and
    # sums exact in FP32
    import torch
    from paper_2605_26016_amd import spx
    rng = np.random.default_rng(9)
    A = rng.integers(-8, 9, (16, 32)).astype(np.float32)
    B = rng.integers(-8, 9, (32, 16)).astype(np.float32)
    D = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    spx.mfma16_probe(to_dev(A), to_dev(B), D)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(D.cpu().numpy(), A @ B)


@pytest.mark.parametrize("L,dil", [((19, 13, 11), (1, 1, 1, 1)), ((21, 17, 10), (1, 2, 4, 8)),
                                   ((5, 3, 2), (1, 2, 4, 8)), ((1, 1, 9), (1, 3, 1, 2))],
                         ids=["d1", "d1248", "tiny_d1248", "line_d1312"])
def test_net_bf16_forward_matches_emulated_oracle(L, dil):
    # the BF16 implicit-GEMM form against the oracle with every layer's
    # weights and inputs rounded as the kernel rounds them (FP32, then BF16)
    # and FP64 sums.  The kernel rounds its FP32 pre-activations and SiLU,
    # summed in the matrix cores' order, to BF16; an activation within a few
    # FP32 ulps of a BF16 rounding boundary can round the other way than the
    # oracle's (one BF16 ulp, 2^-8 relative).  Such a flip moves the outputs
    # of its neighbourhood in the later layers by up to about 2e-3 of max
    # |u| (the bound on every value), and a handful per image touch up to a
    # few tenths of the outputs, so the bulk is checked by the median: the
    # outputs away from flips agree to FP32 accumulation (about 1e-8).  The
    # error against the unrounded FP64 network is printed and bounded
    # loosely (BF16 keeps 8 bits).
    import torch
    from paper_2605_26016_amd import spx
    B = 2
    p32 = init_params(6, scale=1.0)
    Sg, SA, SB, _, t = batch_case(L, B, 60)
    P = L[0] * L[1] * L[2]
    net = spx.Net(dilation=dil)
    spx.net_set_precision(net, "bf16")
    out = torch.zeros((B, 3, P), dtype=torch.float64, device="cuda")
    spx.net_forward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    p64 = p32.astype(np.float64)
    for b in range(B):
        x = oracle_x(Sg[b], SA[b], SB[b], t[b])
        rq = oracle.net_forward(L, p64, x, dil=dil, bf16=True)
        refq, _ = oracle.net_predict_loss(rq, Sg[b])
        r64 = oracle.net_forward(L, p64, x, dil=dil)
        ref64, _ = oracle.net_predict_loss(r64, Sg[b])
        eq = float(np.max(np.abs(got[b] - refq)))
        mdq = float(np.median(np.abs(got[b] - refq)))
        e64 = float(np.max(np.abs(got[b] - ref64)))
        scale = max(1.0, float(np.max(np.abs(rq))))
        print(f"bf16 {L} {dil} image {b}: vs emulated oracle max {eq:.2e} median {mdq:.2e}; vs FP64 net "
              f"max {e64:.2e} (max |u| {np.max(np.abs(r64)):.2f})", flush=True)
        assert eq <= 2e-3 * scale and mdq <= 1e-6 * scale
        assert e64 <= 5e-2 * scale
    # FP32 again after switching back
    spx.net_set_precision(net, "fp32")
    spx.net_forward(net, to_dev(p32), L, B, to_dev(Sg), to_dev(SA), to_dev(SB), to_dev(t), out)
    r64 = oracle.net_forward(L, p64, oracle_x(Sg[0], SA[0], SB[0], t[0]), dil=dil)
    ref64, _ = oracle.net_predict_loss(r64, Sg[0])
    assert np.max(np.abs(out[0].cpu().numpy() - ref64)) <= 1e-5 * max(1.0, float(np.max(np.abs(r64))))


def test_adam_matches_oracle():
    import torch
    from paper_2605_26016_amd import spx
    rng = np.random.default_rng(3)
    n = 1000
    w = rng.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    wd, md, vd = to_dev(w.astype(np.float32)), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    for step in range(1, 6):
        g = rng.standard_normal(n)
        oracle.adam(w, g, m, v, step, lr=1e-2)
        spx.net_adam_step(wd, to_dev(g.astype(np.float32)), md, vd, step, lr=1e-2)
    assert np.max(np.abs(wd.cpu().numpy() - w)) < 1e-5


def test_learned_init_with_zero_net_is_geodesic_and_nonzero_matches_forward():
    import torch
    from paper_2605_26016_amd import spx
    from tests.helpers import gpu_hamiltonian
    from workloads import Workload
    w = Workload(name="t", L=(6, 5, 4), periodic=(0, 0, 0), J_shell=(1.0, 0.188, -0.274, -0.161), field_prec="fp64")
    A, Bv = random_sphere(w.N, 1), random_sphere(w.N, 2)
    n_img = 6
    Y = np.zeros((n_img, 3, w.N))
    Y[0], Y[-1] = A, Bv
    geo = oracle.geodesic_path(A, Bv, n_img)
    net = spx.Net()
    zero = torch.zeros(spx.net_nparams(), dtype=torch.float32, device="cuda")
    Yd = to_dev(Y)
    g = spx.gneb_create([gpu_hamiltonian(w)], [Yd])
    spx.gneb_init_path(g, method=1, net=net, params=zero)
    torch.cuda.synchronize()
    assert np.max(np.abs(Yd.cpu().numpy() - geo)) < 1e-13
    p32 = init_params(5)
    Yd2 = to_dev(Y)
    g2 = spx.gneb_create([gpu_hamiltonian(w)], [Yd2])
    spx.gneb_init_path(g2, method=1, net=net, params=to_dev(p32))
    torch.cuda.synchronize()
    got = Yd2.cpu().numpy()
    p64 = p32.astype(np.float64)
    for n in range(1, n_img - 1):
        tn = np.float32(n / (n_img - 1))
        raw = oracle.net_forward(w.L, p64, oracle_x(geo[n], A, Bv, tn))
        ref, _ = oracle.net_predict_loss(raw, geo[n])
        assert np.max(np.abs(got[n] - ref)) < 1e-5
    assert np.array_equal(got[0], A) and np.array_equal(got[-1], Bv)
    # the same initial path with the network in BF16 on the matrix cores,
    # against the oracle that rounds the same operands to BF16 (a rounding
    # flip moves a raw output by up to a few 1e-3)
    spx.net_set_precision(net, "bf16")
    Yd3 = to_dev(Y)
    g3 = spx.gneb_create([gpu_hamiltonian(w)], [Yd3])
    spx.gneb_init_path(g3, method=1, net=net, params=to_dev(p32))
    torch.cuda.synchronize()
    got = Yd3.cpu().numpy()
    for n in range(1, n_img - 1):
        tn = np.float32(n / (n_img - 1))
        raw = oracle.net_forward(w.L, p64, oracle_x(geo[n], A, Bv, tn), bf16=True)
        ref, _ = oracle.net_predict_loss(raw, geo[n])
        assert np.max(np.abs(got[n] - ref)) < 5e-3
        assert np.max(np.abs(np.sum(got[n] ** 2, axis=0) - 1.0)) < 1e-12
    assert np.array_equal(got[0], A) and np.array_equal(got[-1], Bv)


def test_trained_net_saves_gneb_iterations_at_equal_barrier():
    # the learned part's gain: train the corrector on GNEB-converged
    # skyrmion-annihilation paths (24^2 films) with the library's own kernels,
    # then run GNEB on held-out end states from the geodesic and from the
    # learned initial path; pairs count when both converge to the same barrier
    # (within 0.1 meV); the learned paths must need clearly fewer iterations
    from paper_2605_26016_amd import pathinit
    r = pathinit.learned_vs_geodesic("skyrmion", n_train=60, n_test=6, epochs=150, lr=2e-3, max_iter=20000,
                                     train_sizes=((24, 1.0),), test_sizes=(24, 32), n_img_test=32,
                                     dilation=(1, 1, 1, 1))
    print({k: r[k] for k in ("same_channel_within_0.1meV", "mean_iterations_geodesic_same_channel",
                             "mean_iterations_learned_same_channel", "iteration_ratio_learned_over_geodesic",
                             "train_loss_first_last", "init_ms_test_batch", "init_bf16_vs_fp32_max_dS",
                             "same_channel_bf16_within_0.1meV", "mean_iterations_learned_bf16_same_channel",
                             "seconds")}, flush=True)
    assert r["test_converged_both"] == r["test_paths"]
    assert r["same_channel_within_0.1meV"] >= (2 * r["test_paths"]) // 3
    assert r["train_loss_first_last"][1] < 0.5 * r["train_loss_first_last"][0]
    assert r["iteration_ratio_learned_over_geodesic"] < 0.9
