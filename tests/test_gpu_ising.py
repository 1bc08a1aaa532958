"""End to end from Ising text input on the GPU: read, cluster (host), build
the PEPS, exact-rank boundary MPS, and a frontier-sized merged beam (exact
dynamic programming) must reach the brute-force Ising ground state."""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("kings", [False, True])
def test_ising_file_to_ground_state(tmp_path, kings):
    R, C, t = 2, 3, 2
    n = R * C * t
    rng = np.random.default_rng(7 + kings)
    cl = spg.lattice_clusters(R, C, t)
    # every pair of spins in the same or neighbouring clusters, random J; fields
    def nb(a, b):
        (ra, ca), (rb, cb) = divmod(int(a), C), divmod(int(b), C)
        dr, dc = rb - ra, cb - ca
        return (dr, dc) in ((0, 0), (0, 1), (1, 0)) or (kings and (dr, dc) in ((1, 1), (1, -1)))
    lines = []
    for i in range(n):
        lines.append((i, i, rng.normal()))
        for j in range(i + 1, n):
            if nb(cl[i], cl[j]):
                lines.append((i, j, rng.normal()))
    f = tmp_path / "ising.txt"
    f.write_text("".join(f"{i + 1} {j + 1} {float(v)!r}\n" for i, j, v in lines))
    nn, ii, jj, JJ = spg.read_ising(str(f))
    assert nn == n
    inst = spg.ising_to_potts(nn, ii, jj, JJ, R, C, t, kings, beta=1.0)
    # brute force over all spin configurations
    best = np.inf
    for bits in itertools.product((-1.0, 1.0), repeat=n):
        s = np.array(bits)
        e = np.where(ii == jj, JJ * s[ii], JJ * s[ii] * s[jj]).sum()
        best = min(best, e)
    peps = spg.build_peps(inst)
    env, _ = spg.boundary_mps(peps, 16, want_logZ=False)
    M = inst.d ** (C + 1)
    N = R * C
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    k = spg.branch_and_bound(env, M, st, en, lp, merge_branches=True)
    torch.cuda.synchronize()
    assert k > 0
    assert abs(float(en[0]) - best) < 1e-9
