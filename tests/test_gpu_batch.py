"""Lockstep batches (ks_minimize_batch): every system's run equals its lone ks_minimize bit
for bit — iteration counts, energies and orbital blocks — for mixed grid sizes, orbital
counts (both p_p classes) and storage precisions in one batch."""
import numpy as np
import pytest

from paper_1308_2864_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def ks():
    from paper_1308_2864_amd import ks as _ks
    return _ks


def _specs():
    out = []
    # p = 32 in both precisions: those systems take the Hamiltonian pass that also forms
    # the [X, G] Gram blocks, and form a launch group of their own
    for i, (N, p, M) in enumerate([(16, 3, 2), (24, 12, 4), (20, 17, 5), (16, 32, 6),
                                   (28, 32, 3), (18, 20, 2), (20, 8, 3)]):
        out.append(synth.make_system(N, N, N, 16.0 / (N + 1), p, M, seed=i, cfg="c5",
                                     lo=(-8.0,) * 3, margin=3.0, zrange=(1, 4)))
    return out


def _lone(K, spec, prec, prm):
    s = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD, precision=prec)
    dt = torch.float32 if prec == K.KS_PREC_FP32 else torch.float64
    X = torch.tensor(synth.make_x0(spec, 1), dtype=dt, device="cuda")
    r = s.ks_minimize(X, prm, check=False)
    torch.cuda.synchronize()
    return r, X.cpu().numpy()


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("tau0", [1e-3, 20.0])
def test_batch_equals_lone_runs_bitwise(tau0, graphs):
    """tau0 = 20: first steps far too long, rejected and backtracked (the QR factors queued
    behind each tick's record copy then take the current points' blocks).  graphs: every
    member has graphs enabled, so the ticks are captured per membership and replayed with
    the members' slots read from device memory; the lone runs stay eager."""
    K = ks()
    prm = K.ks_default_params(max_iter=300, tau0=tau0)
    specs = _specs()
    precs = [K.KS_PREC_FP64 if i % 3 else K.KS_PREC_FP32 for i in range(len(specs))]
    systems, blocks = [], []
    for spec, prec in zip(specs, precs):
        systems.append(K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD,
                                          precision=prec))
        if graphs:
            systems[-1].ks_enable_graphs(True)
        dt = torch.float32 if prec == K.KS_PREC_FP32 else torch.float64
        blocks.append(torch.tensor(synth.make_x0(spec, 1), dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    res, codes = K.ks_minimize_batch(systems, blocks, prm)
    torch.cuda.synchronize()
    for i, (spec, prec) in enumerate(zip(specs, precs)):
        assert codes[i] in (K.KS_OK, K.KS_E_NOT_CONVERGED), (i, codes[i])
        r, X = _lone(K, spec, prec, prm)
        assert res[i].iters == r.iters and res[i].nfe == r.nfe, spec.name
        assert res[i].energy == r.energy, spec.name
        assert res[i].hartree_iters_total == r.hartree_iters_total, spec.name
        assert np.array_equal(blocks[i].cpu().numpy(), X), spec.name
        assert res[i].backtracks == r.backtracks, spec.name
    if tau0 > 1.0:
        assert any(x.backtracks > 0 for x in res)


def test_batch_rejects_what_it_cannot_run():
    K = ks()
    spec = _specs()[0]
    ok = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_PCG_FD)
    cg = K.system_from_spec(spec, hartree_solver=K.KS_HARTREE_CG)
    X1 = torch.tensor(synth.make_x0(spec, 1), dtype=torch.float64, device="cuda")
    X2 = X1.clone()
    res, codes = K.ks_minimize_batch([ok, cg], [X1, X2], K.ks_default_params(max_iter=30))
    assert codes[0] in (K.KS_OK, K.KS_E_NOT_CONVERGED)
    assert codes[1] == K.KS_E_UNSUPPORTED
