"""GPU parity of the unique-quartet ERI blocks (mess_eri MESS_ERI_BLOCKS) and
of the deterministic J/K mode.

Blocks: every class's structure-of-arrays region against the oracle's
quartet-list integrals (extended precision), within 1e-12 * max(1, |x|);
classes with many quartets are checked on a seeded sample of them.

Deterministic mode: J and K accumulated exactly in 128-bit fixed point, so
two runs agree bit for bit; the values meet the same bar against the oracle
as the other modes (1e-11 * max(1, |x|)), and an SCF run twice reproduces
every energy and the final density bit for bit.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, random_density, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "water2_spd/0": lambda: G.water_cluster(0, n_waters=2, box=7.0),
    "mol3to20/1004": lambda: G.batched_molecule(1004),
}


def _ncart(l):
    return (l + 1) * (l + 2) // 2


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("tau", [0.0, 1e-10])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eri_blocks(case, tau, prec):
    mess = need_gpu()
    torch = pytest.importorskip("torch")
    mol = CASES[case]()
    B = mess.basis_from_molecule(mol)
    counts, shells = mess.mess_eri_quartets(B, schwarz_tol=tau)
    l = mol.shell_l
    sizes = np.array([_ncart(l[a]) * _ncart(l[b]) * _ncart(l[c]) * _ncart(l[d]) for a, b, c, d in shells])
    p = mess.MESS_FP32 if prec == "fp32" else mess.MESS_FP64
    dt = torch.float32 if prec == "fp32" else torch.float64
    out = torch.zeros(int(sizes.sum()), dtype=dt, device="cuda")
    announce(f"eri blocks {case} tau={tau} {prec}: {int(counts.sum())} quartets, {int(sizes.sum())} integrals")
    mess.mess_eri(B, out, layout=mess.MESS_ERI_BLOCKS, prec=p, schwarz_tol=tau)
    got = host(out).astype(np.float64)
    # every quartet is unique and canonical: pair (ab) >= pair (cd)
    assert len({tuple(q) for q in shells}) == len(shells)
    rng = np.random.Generator(np.random.PCG64(5))
    off, q0 = 0, 0
    worst = 0.0
    for cls in range(21):
        nq = int(counts[cls])
        if nq == 0:
            continue
        blk = shells[q0:q0 + nq]
        nout = int(sizes[q0])
        assert np.all(sizes[q0:q0 + nq] == nout)
        pick = np.sort(rng.choice(nq, size=min(nq, 60), replace=False))
        with core.extended_precision():
            ref = core.eri_quartet_list(mol, blk[pick])
        region = got[off:off + nout * nq].reshape(nout, nq)
        for t, r in zip(pick, ref):
            err = np.abs(region[:, t] - r.reshape(-1)) / np.maximum(1.0, np.abs(r.reshape(-1)))
            worst = max(worst, float(err.max()))
        off += nout * nq
        q0 += nq
    assert off == len(got)
    bar = 1e-4 if prec == "fp32" else 1e-12
    announce(f"  worst relative error {worst:.2e} (bar {bar:g})")
    assert worst < bar
    # a too-small buffer is refused
    small = torch.zeros(8, dtype=dt, device="cuda")
    with pytest.raises(mess.MessError):
        mess.mess_eri(B, small, layout=mess.MESS_ERI_BLOCKS, prec=p, schwarz_tol=tau)


@pytest.mark.parametrize("case", list(CASES))
def test_deterministic_jk_bitwise_and_parity(case):
    mess = need_gpu()
    mol = CASES[case]()
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    D = dev(random_density(N, seed=41))
    runs = []
    for _ in range(2):
        J, K = zeros(N, N), zeros(N, N)
        mess.mess_jk(B, D, J, K, mode=mess.MESS_JK_DETERMINISTIC, schwarz_tol=1e-10)
        runs.append((host(J), host(K)))
    announce(f"deterministic jk {case}: nbf={N}")
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    Jo, Ko, _ = core.jk_unique(mol, G.symmetric_density(N, 41), 1e-10)
    rel = lambda a, b: np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))  # noqa: E731
    assert rel(runs[0][0], Jo) < 1e-11 and rel(runs[0][1], Ko) < 1e-11
    # K alone gives the same bits as K with J
    K2 = zeros(N, N)
    mess.mess_jk(B, D, None, K2, mode=mess.MESS_JK_DETERMINISTIC, schwarz_tol=1e-10)
    assert np.array_equal(host(K2), runs[0][1])


def test_deterministic_scf_reproduces_bitwise():
    mess = need_gpu()
    mol = G.water_cluster(0, n_waters=2, box=7.0)
    traj = []
    for _ in range(2):
        B = mess.basis_from_molecule(mol)
        st = mess.mess_scf_create(B, schwarz_tol=1e-10, conv_tol=1e-9, diis_size=8, deterministic=True)
        es = []
        for _ in range(60):
            e, de, r, c = mess.mess_scf_step(st)
            es.append(e)
            if c:
                break
        assert c
        Dfin = zeros(B.nbf, B.nbf)
        mess.mess_scf_density(st, Dfin)
        traj.append((es, host(Dfin)))
        st.close()
        B.close()
    announce(f"deterministic scf: {len(traj[0][0])} iterations, E = {traj[0][0][-1]:.12f}")
    assert traj[0][0] == traj[1][0]
    assert np.array_equal(traj[0][1], traj[1][1])
    # the same energy as the direct (non-deterministic) SCF
    B = mess.basis_from_molecule(mol)
    st = mess.mess_scf_create(B, schwarz_tol=1e-10, conv_tol=1e-9, diis_size=8)
    for _ in range(60):
        e, de, r, c = mess.mess_scf_step(st)
        if c:
            break
    assert abs(e - traj[0][0][-1]) < 1e-9
