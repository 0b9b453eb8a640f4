"""GPU tests of the operands split into BF16 pieces once per product
(split-precision factorizations whose workspace holds the two pre-split
buffers).  The pieces are the ones the GEMM loaders would form from the FP64
operands, and the MFMAs take them in the same order, so a factorization
through them must equal, to the bit, the same factorization run with a
workspace sized for FP64 (no room for the buffers, so the loaders split the
operands themselves).  Shapes span 64 x 64 and 128 x 128 product tiles, a
ragged last block and the sampling products' split-K, 1 to 45 partials.  The oracle parity of
these paths is covered by test_gpu_split_oracle and test_gpu_factor."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_00998_amd import binding
    binding.lib()
    return binding


CASES = [  # m, n, b, q, prec
    (1100, 900, 64, 1, "bf16x3"),
    (1100, 900, 96, 1, "bf16x3_bf16x6"),
    (2600, 2600, 128, 1, "bf16x3_bf16x6"),
    (2600, 2500, 128, 2, "bf16x3_fp32"),
    (3000, 2000, 256, 1, "bf16x3"),
    # thin samples of a tall matrix: the sampling products' split-K takes 8
    # partials in the first steps, then deep splits of 19 to 45 once the
    # sample has at most 32 output tiles, and the row count leaves a ragged
    # last chunk of 8 in the reduction
    (5004, 3000, 64, 1, "bf16x3_bf16x6"),
]


@pytest.mark.parametrize("m,n,b,q,prec", CASES)
def test_presplit_path_equals_loader_split(B, m, n, b, q, prec):
    from paper_1703_00998_amd import workloads as wl
    print(f"presplit {prec} {m}x{n} b={b} q={q}", flush=True)
    sig = np.exp(-np.arange(1, min(m, n) + 1) / (0.25 * min(m, n)))
    A = wl.planted(m, n, sig, seed=m + n + b)
    G = wl.gaussian_g(m, n, b, seed=7)
    dG = B.colmajor(G)
    full = B.workspace_size(m, n, b, q, prec, True, True)
    base = B.workspace_size(m, n, b, q, "fp64", True, True)
    assert full > base  # room for the two pre-split buffers
    outs = []
    for nbytes in (full, base):
        T = B.colmajor(A)
        U, V = B.empty_colmajor(m, m), B.empty_colmajor(n, n)
        ws = B.workspace(nbytes)
        wp, _ = B._aligned_ptr(ws)
        k = ctypes.c_int64(0)
        # Through the C ABI with exactly nbytes of workspace (the binding
        # would refuse the FP64-sized one for a split-precision call).
        st = B.lib().randutv_factor(m, n, b, q, B._ptr(T), m, B._ptr(dG), m, B._ptr(U), m,
                                    B._ptr(V), n, 0, 0.0, B.PREC[prec], B.FORM_U | B.FORM_V,
                                    wp, nbytes, ctypes.byref(k), B._stream())
        assert st == 0, st
        torch.cuda.synchronize()
        outs.append((k.value, T.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()))
    (k1, T1, U1, V1), (k2, T2, U2, V2) = outs
    assert k1 == k2 == min(m, n)
    np.testing.assert_array_equal(T1, T2)
    np.testing.assert_array_equal(U1, U2)
    np.testing.assert_array_equal(V1, V2)
    res = np.linalg.norm(A - U1 @ T1 @ V1.T) / np.linalg.norm(A)
    assert res < 1e-5, res
