"""rmc_kron_apply_noalloc (the entry point that allocates nothing) against
rmc_kron_apply on the same inputs, through the C ABI, on the GPU: two calls in a row
(the second with a smaller coupling and fewer vectors) in every precision, to the same
tolerances as the Kronecker matvec parity tests (FP64 1e-12, FP32 2e-5, BF16 3e-2 of the
output scale); the context's arena is untouched; a coupling whose scratch exceeds the
fixed array is refused with RMC_ERR_ARG."""
import numpy as np
import pytest

from oracle import recursion as OR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2609_02394_amd import rmc

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = rmc.Context(arena_bytes=1 << 30)
    yield c
    c.close()


def _module(ctx, rng, k):
    E = np.sort(rng.uniform(-3.0, 0.0, k))
    ops, mats = [], {}
    for s, o in [(0, "Z"), (0, "X"), (0, "T"), (7, "Z"), (7, "X"), (7, "T")]:
        M = rng.standard_normal((k, k))
        M = (M - M.T) if o == "T" else (M + M.T)
        M /= np.linalg.norm(M, 2)
        ops.append((s, o, M))
        mats[(s, o)] = M
    return ctx.module_import(8, E, ops, dim=4 * k), E, mats


def _case(ctx, rng, kA, kB, T):
    A, EA, mA = _module(ctx, rng, kA)
    B, EB, mB = _module(ctx, rng, kB)
    keys = [(7, "X"), (7, "T"), (7, "Z")][:T]
    keysB = [(0, "X"), (0, "T"), (0, "Z")][:T]
    coefs = [0.25, -0.25, 0.3][:T]
    idA = A.project_ops([s for s, _ in keys], [o for _, o in keys])
    idB = B.project_ops([s for s, _ in keysB], [o for _, o in keysB])
    H = OR.effective_hamiltonian(EA, EB, [(c, mA[a], mB[b]) for c, a, b in zip(coefs, keys, keysB)])
    return A, B, coefs, idA, idB, H


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
def test_noalloc_kron_apply_equals_kron_apply_twice(ctx, prec):
    import torch

    print("[case] kron_apply_noalloc", prec, flush=True)
    rng = np.random.default_rng(2609 + prec)
    tol = {0: 1e-12, 1: 2e-5, 2: 3e-2}[prec]
    for (kA, kB, T, nv) in [(96, 80, 3, 9), (40, 24, 2, 3)]:  # the second call is smaller
        A, B, coefs, idA, idB, H = _case(ctx, rng, kA, kB, T)
        X = torch.tensor(rng.standard_normal((nv, kA * kB)), device="cuda")
        Y_ref = ctx.kron_apply(A, B, coefs, idA, idB, X, prec).cpu().numpy()
        used = ctx.arena_usage()
        Y = torch.full_like(X, float("nan"))
        ctx.kron_apply_noalloc(A, B, coefs, idA, idB, X, Y, prec)
        Y = Y.cpu().numpy()
        assert ctx.arena_usage() == used
        scale = np.max(np.abs(Y_ref))
        assert np.all(np.isfinite(Y))
        assert np.max(np.abs(Y - Y_ref)) <= tol * scale, (kA, kB, T, prec)
        # both against the explicit Kronecker sum of the oracle
        ref = X.cpu().numpy() @ H.T
        assert np.max(np.abs(Y - ref)) <= tol * np.max(np.abs(ref))
        A.free()
        B.free()


def test_noalloc_kron_apply_refuses_what_does_not_fit(ctx):
    import torch

    from paper_2609_02394_amd import rmc

    print("[case] kron_apply_noalloc too large", flush=True)
    rng = np.random.default_rng(7)
    A, _, _ = _module(ctx, rng, 192)
    B, _, _ = _module(ctx, rng, 192)
    ia = A.project_ops([7, 7, 7], ["X", "T", "Z"])
    ib = B.project_ops([0, 0, 0], ["X", "T", "Z"])
    coefs = [0.1] * 8
    opA = [ia[i % 3] for i in range(8)]
    opB = [ib[i % 3] for i in range(8)]
    X = torch.zeros((1, 192 * 192), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(rmc.RmcError) as ei:
        ctx.kron_apply_noalloc(A, B, coefs, opA, opB, X, Y, 1)
    assert ei.value.status == rmc.ERR_ARG
    A.free()
    B.free()
