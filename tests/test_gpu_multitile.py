"""The persistent convolution kernels on grids with more tiles than resident
blocks, so that every block walks several tiles (the tile loop, the next-tile
prefetch and the LDS reuse between tiles), and the preconditioner with
full-width He-initialised weights at the bench's 256 x 256 size, against the
oracle.  At B = 4 and 256 x 256 a level-0 layer has 1024 16 x 16 tiles (1444
14 x 14 residual-block tiles), several per block at the occupancy of these
kernels on 256 compute units."""
import numpy as np
import pytest
import torch

import bf16_storage as B
from helpers import f32, medium, rand_c, relerr
from oracle import operator as op
from oracle import unet as U
from paper_2405_17696_amd import api, synth

pytestmark = pytest.mark.gpu

CK_PERS = 0     # the persistent halo kernel's id for helm_conv_force
CK_DL64 = 10    # the double-buffered direct-load kernel, one 16 x 32 tile per block
CK_GPF64, CK_GPF128 = 12, 13   # the implicit GEMM with three chunks in flight (64 x 64, 64 x 128 tiles)


def bf(x):
    return B.bf16(x)


def rnd(shape, seed, scale=1.0):
    return bf(scale * np.random.default_rng(seed).standard_normal(shape))


@pytest.mark.parametrize("ck,c1,c2,bcast,cout", [(CK_PERS, 32, 0, False, 32), (CK_PERS, 32, 32, True, 32)])
def test_persistent_conv_many_tiles_per_block(gpu, ck, c1, c2, bcast, cout):
    Bn, H, W_ = 4, 256, 256
    print("persistent conv multi-tile kernel", ck, "c1", c1, "c2", c2, "cout", cout, flush=True)
    x1 = rnd((Bn, H, W_, c1), 31)
    x2 = rnd((1, H, W_, c2), 32) if c2 else None
    Wt = rnd((cout, 3, 3, c1 + c2), 33, scale=np.sqrt(2.0 / (9 * (c1 + c2))))
    b = rnd((cout,), 34, 0.1)
    api.helm_conv_force(ck)
    try:
        y = api.cnn_layer_forward(0, 1, x1, Wt, b, x2=x2, bcast2=bcast, relu=True)
    finally:
        api.helm_conv_force(-1)
    x = x1 if x2 is None else np.concatenate([x1, np.broadcast_to(x2, x1.shape[:3] + x2.shape[3:])], axis=-1)
    ref = np.maximum(U.conv3x3(x, Wt, b, 1), 0)
    e = relerr(y, ref)
    print("rel err", e)
    assert e <= 1e-5
    # every sample and every tile row/column is covered (a skipped tile leaves zeros or stale values)
    for s in range(Bn):
        for t in range(0, H, 16):
            assert relerr(y[s, t:t + 16], ref[s, t:t + 16]) <= 1e-5


@pytest.mark.parametrize("c2,bcast,cout,use_resid", [(0, False, 64, False), (64, True, 64, False),
                                                     (0, False, 128, True)])
def test_direct_load_conv_many_tiles(gpu, c2, bcast, cout, use_resid):
    """The direct-load kernel on 64-channel layers (plain, concatenated broadcast
    context, 128 outputs with a residual) over 9 samples of 128 x 128: 288 tiles
    of 16 x 32, more than can be resident at once."""
    Bn, H, W_ = 9, 128, 128
    ck = CK_DL64
    print("direct-load conv, c2", c2, "cout", cout, flush=True)
    x1 = rnd((Bn, H, W_, 64), 51)
    x2 = rnd((1, H, W_, c2), 52) if c2 else None
    Wt = rnd((cout, 3, 3, 64 + c2), 53, scale=np.sqrt(2.0 / (9 * (64 + c2))))
    b = rnd((cout,), 54, 0.1)
    resid = rnd((Bn, H, W_, cout), 55) if use_resid else None
    api.helm_conv_force(ck)
    try:
        y = api.cnn_layer_forward(0, 1, x1, Wt, b, x2=x2, bcast2=bcast, resid=resid, relu=not use_resid)
    finally:
        api.helm_conv_force(-1)
    x = x1 if x2 is None else np.concatenate([x1, np.broadcast_to(x2, x1.shape[:3] + x2.shape[3:])], axis=-1)
    ref = U.conv3x3(x, Wt, b, 1)
    ref = ref + resid if use_resid else np.maximum(ref, 0)
    e = relerr(y, ref)
    print("rel err", e)
    assert e <= 1e-5
    for s in range(Bn):
        for t in range(0, H, 16):
            assert relerr(y[s, t:t + 16], ref[s, t:t + 16]) <= 1e-5


def test_fused_resblock_many_tiles_per_block(gpu):
    Bn, H, W_ = 4, 256, 256
    print("resblock multi-tile", flush=True)
    x = rnd((Bn, H, W_, 32), 41)
    W1 = rnd((32, 3, 3, 32), 42, scale=np.sqrt(2.0 / 288))
    W2 = rnd((32, 3, 3, 32), 43, scale=np.sqrt(2.0 / 288))
    b1 = rnd((32,), 44, 0.1)
    b2 = rnd((32,), 45, 0.1)
    y = api.cnn_layer_resblock(x, W1, b1, W2, b2)
    h = bf(np.maximum(U.conv3x3(x, W1, b1, 1), 0))
    ref = x + U.conv3x3(h, W2, b2, 1)
    e = relerr(y, ref)
    print("rel err", e)
    assert e <= 5e-3                                      # output stored in BF16
    for s in range(Bn):
        for t in range(0, H, 14):
            assert relerr(y[s, t:t + 14], ref[s, t:t + 14]) <= 5e-3


def test_precond_apply_full_width_full_size(gpu):
    """M_net(r) at 256 x 256, batch 2, default widths, He-normal weights at full
    scale (no damped head) and small random biases: the inference path with the
    fused first layer + context convolution and the fused residual blocks, over
    1024 level-0 tiles per launch; with the built-in kernel choice and with the
    64-channel layers pinned to the direct-load kernel."""
    med, _ = synth.config2_medium()
    k2, gam = f32(med.kappa2), f32(med.gamma)
    widths = (32, 64, 128, 256)
    layers = U.all_layers(widths, 2)
    theta = U.init_params(layers, np.random.default_rng(51)).astype(np.float32)
    o = 0
    rng = np.random.default_rng(52)
    for l in layers:
        o += int(np.prod(l.wshape()))
        theta[o:o + l.cout] = 0.05 * rng.standard_normal(l.cout)
        o += l.cout
    net = api.cnn_create(widths, seed=0, down_res=2)
    api.cnn_set_params(net, theta)
    theta = theta.astype(np.float64)
    H = api.helm_setup(torch.tensor(k2, dtype=torch.float32, device="cuda"),
                       torch.tensor(gam, dtype=torch.float32, device="cuda"), med.omega, med.h)
    r = rand_c((2, 256, 256), 53).astype(np.complex64)
    # the built-in kernel choice, then the 64-channel layers on the direct-load kernel (its bf16
    # outputs leave through the LDS epilogue)
    outs = {}
    try:
        for ck in (-1, CK_DL64):
            print("precond apply full size, kernel", ck, flush=True)
            api.helm_conv_force(ck)
            outs[ck] = api.cnn_precond_apply(net, H, torch.tensor(r, device="cuda")).cpu().numpy()
    finally:
        api.helm_conv_force(-1)
    e = outs[-1]
    rr = r.astype(np.complex128)
    ref = U.cnn_precond(theta, k2, gam, med.omega, med.h, med.h, rr, widths, 2)
    orig = U.Net
    U.Net = B.Bf16Net
    try:
        emu = U.cnn_precond(theta, k2, gam, med.omega, med.h, med.h, rr, widths, 2)
    finally:
        U.Net = orig
    e64, eb = relerr(e, ref), relerr(e, emu)
    print("rel err vs FP64", e64, "vs BF16-storage oracle", eb, "floor", relerr(emu, ref))
    # BF16 storage alone moves this network's output by 1.2% on this case
    # (the BF16-storage oracle above); P7's 2e-2 bound
    assert e64 <= 2e-2
    for s in range(2):
        assert relerr(e[s], ref[s]) <= 2e-2
    for ck in (CK_DL64,):
        print("kernel", ck, "rel err vs FP64", relerr(outs[ck], ref), "vs BF16-storage oracle", relerr(outs[ck], emu))
        for s in range(2):
            assert relerr(outs[ck][s], ref[s]) <= 2e-2



def test_forced_kernels_in_a_masked_solve(gpu):
    """CNN-FGMRES(10) at 128 x 128 on right-hand sides that converge at
    different iterations, so that the convolution kernels skip the finished
    ones' tiles through the per-RHS flags, with the 64-channel layers on the
    built-in choice and on the direct-load kernel: the kernels add the same
    products in the same order, so iteration counts and solutions agree."""
    n = 128
    med = medium(n, n, seed=21)
    H = api.helm_setup(torch.tensor(med.kappa2, dtype=torch.float32, device="cuda"),
                       torch.tensor(med.gamma, dtype=torch.float32, device="cuda"), med.omega, med.h)
    net = api.cnn_create(seed=1)
    b = np.zeros((5, n, n), np.complex128)
    b[0] = rand_c((n, n), 61)
    b[1, n // 2, n // 2] = 1.0
    b[2, 10, 17] = 1.0
    b[3] = rand_c((n, n), 62)
    b[4] = 0.5 * (b[0] + b[1])
    bt = torch.tensor(b.astype(np.complex64), device="cuda")
    api.helm_autotune(0)                                 # the built-in choice, not a timed one
    res = {}
    try:
        for ck in (-1, CK_DL64):
            print("masked solve, kernel", ck, flush=True)
            api.helm_conv_force(ck)
            x, it, rr, st, code = api.helm_solve(H, bt, tol=1e-6, precond="cnn_vu", maxit=600, net=net, restart=10)
            assert code == 0 and np.all(st == 0)
            res[ck] = (x.cpu().numpy(), it)
            print("iterations", it, flush=True)
    finally:
        api.helm_conv_force(-1)
        api.helm_autotune(1)                             # the library's default
    x0, it0 = res[-1]
    assert it0.max() > it0.min()                          # finished right-hand sides are masked for a while
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    for ck, (x, it) in res.items():
        assert np.all(np.abs(it - it0) <= 1)
        assert relerr(x, x0) <= 1e-5
        assert np.all(op.relres(coef, x, b, med.h, med.h) <= 1e-6)


@pytest.mark.parametrize("precond,use_graph,nops", [("cnn_vu", False, 1), ("cnn_vu", True, 1), ("cnn", False, 1),
                                                    ("cnn_vu", False, 2), ("cnn_vu", True, 2)])
def test_two_stream_preconditioner_matches_one_stream(gpu, precond, use_graph, nops):
    """streams=2 applies the network (and for M_VU its residual and V-cycle) to
    the two halves of each operator's batch on two streams, also inside a
    captured restart cycle: one operator (3 + 2 right-hand sides) or two
    (groups of 3 and 2, split 2 + 1 and 1 + 1).  Every right-hand side sees the
    same arithmetic as with one stream, so iterations and solutions agree."""
    n = 128
    med = medium(n, n, seed=23)
    k2 = torch.tensor(med.kappa2, dtype=torch.float32, device="cuda")
    gm = torch.tensor(med.gamma, dtype=torch.float32, device="cuda")
    H = api.helm_setup(k2, gm, med.omega, med.h)
    ops = [H] if nops == 1 else [H, api.helm_setup(k2, gm, 0.8 * med.omega, med.h)]
    rhs_op = None if nops == 1 else [0, 0, 0, 1, 1]
    net = api.cnn_create(seed=1)
    b = np.zeros((5, n, n), np.complex128)
    b[0] = rand_c((n, n), 71)
    b[1, n // 3, n // 2] = 1.0
    b[2] = rand_c((n, n), 72)
    b[3, 5, 9] = 1.0
    b[4] = 0.3 * b[0] + b[3]
    bt = torch.tensor(b.astype(np.complex64), device="cuda")
    maxit = 600 if precond == "cnn_vu" else 30
    api.helm_autotune(0)
    try:
        out = {}
        for streams in (1, 2):
            print(precond, "graph", use_graph, "streams", streams, flush=True)
            x, it, rr, st, code = api.helm_solve(ops, bt, tol=1e-6, precond=precond, maxit=maxit, net=net, restart=10,
                                                 use_graph=use_graph, streams=streams, rhs_op=rhs_op)
            out[streams] = (x.cpu().numpy(), it, rr)
            print("iterations", it, flush=True)
    finally:
        api.helm_autotune(1)
    (x1, it1, rr1), (x2, it2, rr2) = out[1], out[2]
    assert np.array_equal(it1, it2)
    assert np.array_equal(rr1, rr2)
    assert relerr(x2, x1) <= 1e-12
    if precond == "cnn_vu":
        coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
        sel = slice(0, 5) if nops == 1 else slice(0, 3)
        assert np.all(op.relres(coef, x2[sel], b[sel], med.h, med.h) <= 1e-6)
    with pytest.raises(Exception):
        api.helm_solve(H, bt, tol=1e-6, precond=precond, maxit=5, net=net, streams=3)


@pytest.mark.parametrize("ck,H,cin,cout", [(CK_GPF64, 256, 32, 64), (CK_GPF128, 128, 64, 128)])
def test_prefetch_gemm_stride2_full_size(gpu, ck, H, cin, cout):
    """The stride-2 layers the autotuner gives to the implicit GEMM with three
    chunks in flight, at the network's sizes (B = 4: 1024 and 256 tiles of 64
    output pixels; 9 and 18 chunks of 32 channels), against the oracle."""
    Bn = 4
    print("prefetch GEMM stride 2, kernel", ck, "input", H, cin, "->", cout, flush=True)
    x = rnd((Bn, H, H, cin), 81)
    Wt = rnd((cout, 3, 3, cin), 82, scale=np.sqrt(2.0 / (9 * cin)))
    b = rnd((cout,), 83, 0.1)
    api.helm_conv_force(ck)
    try:
        y = api.cnn_layer_forward(0, 2, x, Wt, b, relu=True)
    finally:
        api.helm_conv_force(-1)
    ref = np.maximum(U.conv3x3(x, Wt, b, 2), 0)
    e = relerr(y, ref)
    print("rel err", e)
    assert e <= 1e-5
    for s in range(Bn):
        assert relerr(y[s], ref[s]) <= 1e-5
