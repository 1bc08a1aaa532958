"""The reduced-precision form of the boundary MPS's GEMMs (spg_set_gemm_precision:
FP32 operands and FP32 accumulation on the matrix cores, FP64 results; QR, SVD
and the MPO d-index contractions stay FP64), through the C ABI.

Where nothing is truncated (strips at their exact Schmidt ranks, the king's
strips at the config-2 distributions among them) the contraction stays exact up
to the products' rounding: each GEMM output carries a relative error of at most
about K * 2^-24 (K <= 64 here, 4e-6), and the row functions' norms multiply such
errors over a few products per site, so log Z moves by far less than 1e-5
(measured: at most 3e-7) and every row function keeps its direction to 1e-10
(measured: 4e-12).  The test pins that, and that the FP64 default is restored.
At the truncated workloads the form is measured by the bench
(forms.boundary_mps_fp32_products), not pinned: it does not keep the
contraction valid there."""
import numpy as np
import pytest

from workloads import random_potts, spin_instance, potts_from_spins

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402
from oracle.exact import row_transfer  # noqa: E402


def _cases():
    out = []
    for R, C in ((4, 3), (6, 3)):
        si = spin_instance(R, C, 4, True, 0, h=("normal", 1.0), j_in=("normal", 1.0),
                           j_out=("normal", 1.0))
        out.append((f"kings{R}x{C}_d16_beta2", potts_from_spins(si, beta=2.0), 16))
    out.append(("rand4x4_d4", random_potts(4, 4, 4, True, seed=44, beta=0.9), 16))
    out.append(("rand3x4_d8", random_potts(3, 4, 8, True, seed=45, beta=0.7), 64))
    return out


CASES = _cases()


def _rows_and_logz(inst, chi, fp32):
    spg.set_gemm_precision(fp32)
    try:
        env, lz = spg.boundary_mps(spg.build_peps(inst), chi)
        torch.cuda.synchronize()
    finally:
        spg.set_gemm_precision(False)
    T, _ = spg.env_export(env)
    return spg.unpack_mps(T, spg.env_info(env).bond_dims), lz


def _dense(row):
    t = row[0][0]
    for A in row[1:]:
        t = np.tensordot(t, A, axes=([t.ndim - 1], [0]))
    return t[..., 0].ravel()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp32_products_exact_rank(case):
    name, inst, chi = case
    print(f"fp32 products {name}", flush=True)
    logs, lz_exact = row_transfer(inst, max_row_states=1 << 21)
    rows, lz = _rows_and_logz(inst, chi, True)
    assert abs(lz - lz_exact) <= 1e-5, (lz, lz_exact)
    for r in range(inst.rows):
        a = _dense(rows[r])
        b = np.exp(logs[r] - logs[r].max()).ravel()
        ov = abs(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
        assert 1.0 - ov <= 1e-10, (r, ov)
    # the default (FP64 products) is back: the same call is exact to rounding
    _, lz64 = _rows_and_logz(inst, chi, False)
    assert abs(lz64 - lz_exact) <= 1e-9 * abs(lz_exact)


def test_gemm_precision_rejects_other_values():
    with pytest.raises(spg.SpgError):
        spg._check(spg.load().spg_set_gemm_precision(2))
