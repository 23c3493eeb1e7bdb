"""Slice stacks: S images sharing one 2D matrix, one sparse-times-dense
product per subset (slices as columns), optional axial penalty."""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402
from paper_2106_03172_amd import binding  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("S,axial", [(5, True), (70, True), (3, False)])
def test_stack_matches_oracle(S, axial):
    """OSEM then SVREM on a stack (S = 70 spans two 64-slice chunks with a
    ragged tail) against the FP64 oracle's multi-slice model."""
    P = datagen.make_multislice_problem(40, 40, 2.5, 36, 55, 2.5, 6, 2e4 * S, n_slices=S, seed=S)
    Ao = oracle.system_matrix(P.geom)
    beta = 5e-2
    m = oracle.Model(Ao, P.g, P.w, P.geom, 6, beta=beta, axial=axial)
    A = pkg.SystemMatrix(P.geom, 6)
    f0 = np.ones((S, P.geom.n_pixels))
    flags = binding.FLAG_AXIAL_PENALTY if axial else 0
    R = pkg.Recon(A, P.g, P.w, f0, pkg.params("svrem", alpha=0.7, eta=1, beta=beta, flags=flags))
    R.osem_epoch(list(range(6)))
    fo = oracle.osem_epoch(m, f0, range(6))
    assert rel(R.image().cpu().numpy(), fo) <= 1e-5
    alg = oracle.SVREM(m, fo, 0.7, 1)
    for e in range(3):
        o = datagen.make_order(6, 6, seed=60 + e)
        R.svrem_epoch(o)
        alg.run(o)
        assert rel(R.image().cpu().numpy(), alg.f) <= 1e-5
    phi = R.objective()
    assert abs(phi - m.objective(R.image().cpu().numpy().astype(np.float64))) <= 1e-6 * abs(phi)


def test_stack_checkpoint_and_determinism():
    S = 9
    P = datagen.make_multislice_problem(32, 32, 2.5, 30, 45, 2.5, 5, 1e5, n_slices=S, seed=2)
    A = pkg.SystemMatrix(P.geom, 5)
    f0 = np.ones((S, P.geom.n_pixels))
    prm = pkg.params("svrem", alpha=0.7, eta=2, beta=1e-2, flags=binding.FLAG_AXIAL_PENALTY)
    orders = [datagen.make_order(5, 5, seed=80 + e) for e in range(4)]

    def run(cut=None):
        R = pkg.Recon(A, P.g, P.w, f0, prm)
        R.osem_epoch(list(range(5)))
        for e, o in enumerate(orders):
            if e == cut:
                st = R.get_state()
                R = pkg.Recon(A, P.g, P.w, f0, prm)
                R.set_state(st)
            R.svrem_epoch(o)
        return R.image().cpu().numpy()

    a = run()
    np.testing.assert_array_equal(a, run())
    np.testing.assert_array_equal(a, run(cut=2))


def test_stack_rejects_gradient_algorithms():
    P = datagen.make_multislice_problem(16, 16, 2.5, 12, 23, 2.5, 3, 1e4, n_slices=3, seed=1)
    A = pkg.SystemMatrix(P.geom, 3)
    with pytest.raises(pkg.SvrError):
        pkg.Recon(A, P.g, P.w, np.ones((3, 256)), pkg.params("saga"))


def test_stack_beyond_32bit_offsets_is_rejected():
    """A stack whose image block passes 2^31 bytes is refused at creation,
    before the (small, valid) data pointers are read."""
    P = datagen.make_multislice_problem(16, 16, 2.5, 12, 23, 2.5, 3, 1e4, n_slices=2, seed=1)
    A = pkg.SystemMatrix(P.geom, 3)
    t = torch.ones(1024, device="cuda")
    S = (2 ** 31) // (4 * A.N) + 1
    with pytest.raises(pkg.SvrError, match="too large"):
        binding.svr_recon_create(A.h, t, t, t, S, pkg.params("svrem"))


def _bf16_weights(A):
    """The FP64 lengths rounded as the library stores BF16 weights: to FP32,
    then to BF16 with round-to-nearest-even (test-side rounding of the
    oracle's own matrix)."""
    u = np.asarray(A.data, np.float32).view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    B = A.copy()
    B.data = r.view(np.float32).astype(np.float64)
    return B


@pytest.fixture(scope="module")
def full_stack():
    cfg = datagen.CONFIG_MULTISLICE
    P = datagen.make_multislice_problem(cfg["nx"], cfg["ny"], cfg["pixel_mm"], cfg["n_views"], cfg["n_bins"],
                                        cfg["bin_mm"], cfg["n_subsets"], cfg["counts"], n_slices=cfg["n_slices"],
                                        seed=cfg["seed"])
    Ao = oracle.system_matrix(P.geom)
    return cfg, P, Ao


@pytest.mark.parametrize("wtype", [pkg.SVR_W_F32, pkg.SVR_W_BF16])
def test_full_size_stack_sampled_slices(full_stack, wtype):
    """127 slices of 285 x 285 (2.5 mm), 344 views x 435 bins, 21 subsets,
    in-plane penalty only, so slices are independent: sampled slices of the
    GPU stack after OSEM and 3 SVREM calls (6 epochs) are compared with
    single-slice oracle runs of the same data.  BF16 weights are compared with
    the oracle run on the same BF16-rounded lengths (parity bar), and with the
    exact lengths (the precision cost, about 1e-3)."""
    cfg, P, Ao = full_stack
    Ns, S = cfg["n_subsets"], cfg["n_slices"]
    A = pkg.SystemMatrix(P.geom, Ns, wtype)
    beta = 1e-3
    f0 = np.ones((S, P.geom.n_pixels))
    R = pkg.Recon(A, P.g, P.w, f0, pkg.params("svrem", alpha=0.7, eta=1, beta=beta))
    R.osem_epoch(list(range(Ns)))
    orders = [datagen.make_order(Ns, Ns, seed=90 + c) for c in range(3)]
    for o in orders:
        R.svrem_epoch(o)
    fg = R.image().cpu().numpy()
    Aw = Ao if wtype == pkg.SVR_W_F32 else _bf16_weights(Ao)
    sample = [0, 63, 126]
    errs = []
    for Am in ((Aw,) if wtype == pkg.SVR_W_F32 else (Aw, Ao)):
        # the sampled slices as a 3-slice stack without axial coupling: each
        # slice runs exactly as alone
        m = oracle.Model(Am, P.g[sample], P.w[sample], P.geom, Ns, beta=beta)
        alg = oracle.SVREM(m, oracle.osem_epoch(m, np.ones((3, P.geom.n_pixels)), range(Ns)), 0.7, 1)
        for o in orders:
            alg.run(o)
        errs.append([rel(fg[sl], alg.f[i]) for i, sl in enumerate(sample)])
    print(f"wtype {wtype} slices {sample}: rel L2 {errs}", flush=True)
    assert max(errs[0]) <= 1e-5
    if len(errs) > 1:
        assert max(errs[1]) <= 2.5e-3


@pytest.mark.parametrize("wtype", [pkg.SVR_W_F32, pkg.SVR_W_BF16])
def test_axial_stack_at_full_in_plane_size(full_stack, wtype):
    """The stack's in-plane size (285 x 285, 344 x 435, 21 subsets) with the
    8 + 2 axial penalty, on the first 6 slices (the axial coupling makes every
    slice depend on all others, so the oracle runs the whole stack): OSEM and
    3 SVREM calls (6 epochs) against the oracle, every call."""
    cfg, P, Ao = full_stack
    Ns, S = cfg["n_subsets"], 6
    g, w = P.g[:S], P.w[:S]
    A = pkg.SystemMatrix(P.geom, Ns, wtype)
    beta = 1e-3
    f0 = np.ones((S, P.geom.n_pixels))
    R = pkg.Recon(A, g, w, f0, pkg.params("svrem", alpha=0.7, eta=1, beta=beta, flags=binding.FLAG_AXIAL_PENALTY))
    Aw = Ao if wtype == pkg.SVR_W_F32 else _bf16_weights(Ao)
    m = oracle.Model(Aw, g, w, P.geom, Ns, beta=beta, axial=True)
    R.osem_epoch(list(range(Ns)))
    alg = oracle.SVREM(m, oracle.osem_epoch(m, f0, range(Ns)), 0.7, 1)
    for c in range(3):
        o = datagen.make_order(Ns, Ns, seed=120 + c)
        R.svrem_epoch(o)
        alg.run(o)
        e = rel(R.image().cpu().numpy(), alg.f)
        print(f"wtype {wtype} axial call {c}: rel L2 {e:.2e}", flush=True)
        assert e <= 1e-5, (c, e)
    phi = R.objective()
    assert abs(phi - m.objective(R.image().cpu().numpy().astype(np.float64))) <= 1e-6 * abs(phi)


@pytest.mark.parametrize("wtype", [pkg.SVR_W_F32, pkg.SVR_W_BF16])
def test_axial_stack_twenty_epochs(full_stack, wtype):
    """The stack's configuration over its stated horizon: SVREM for 20 epochs
    (10 calls of an anchor and 21 subset updates) with the 8 + 2 axial penalty,
    on the first 10 slices of the 285 x 285 / 344 x 435 / 21-subset stack,
    against the oracle after every call (BF16 weights against the oracle on the
    same BF16-rounded lengths)."""
    cfg, P, Ao = full_stack
    Ns, S = cfg["n_subsets"], 10
    g, w = P.g[:S], P.w[:S]
    A = pkg.SystemMatrix(P.geom, Ns, wtype)
    beta = 1e-3
    f0 = np.ones((S, P.geom.n_pixels))
    R = pkg.Recon(A, g, w, f0, pkg.params("svrem", alpha=0.7, eta=1, beta=beta, flags=binding.FLAG_AXIAL_PENALTY))
    Aw = Ao if wtype == pkg.SVR_W_F32 else _bf16_weights(Ao)
    m = oracle.Model(Aw, g, w, P.geom, Ns, beta=beta, axial=True)
    R.osem_epoch(list(range(Ns)))
    alg = oracle.SVREM(m, oracle.osem_epoch(m, f0, range(Ns)), 0.7, 1)
    worst = 0.0
    for c in range(10):
        o = datagen.make_order(Ns, Ns, seed=200 + c)
        R.svrem_epoch(o)
        alg.run(o)
        e = rel(R.image().cpu().numpy(), alg.f)
        worst = max(worst, e)
        assert e <= 1e-5, (c, e)
    print(f"wtype {wtype}: 20 epochs, worst rel L2 {worst:.2e}", flush=True)
    phi = R.objective()
    assert abs(phi - m.objective(R.image().cpu().numpy().astype(np.float64))) <= 1e-6 * abs(phi)
