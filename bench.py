#!/usr/bin/env python3
"""Benchmark of the Hartree-Fock hot path on one MI355X.

One step = one complete closed-shell SCF of the 60-atom water-cluster
workload (300 Cartesian s/p/d functions, Schwarz threshold 1e-10): basis
creation (normalisation, primitive pairs, Schwarz factors), unique
shell-quartet work lists, one-electron integrals, overlap eigensolve and
orthogonaliser, core-Hamiltonian guess, then Fock builds with direct J/K
(ERI class kernels), Pulay DIIS and purification until |dE| < 1e-8 Ha.

Prints one JSON line (stdout).  value = shell quartets evaluated per second
over the timed steps (all Fock builds); the roofline block is for the
dominant ERI class kernel, from HIP events recorded on the launch stream
around every class launch inside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop/FMA x 2.4 GHz
CLASS_NAMES = {}
_PC = ["ss", "ps", "pp", "ds", "dp", "dd"]
for _cb in range(6):
    for _ck in range(_cb + 1):
        CLASS_NAMES[_cb * (_cb + 1) // 2 + _ck] = f"({_PC[_cb]}|{_PC[_ck]})"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name, seed):
    from mess_inputs import generators as G
    if name == "water60_spd":
        return G.water_cluster(seed)
    if name == "hco6_sp":
        return G.random_small_molecule(seed)
    raise SystemExit(f"unknown workload {name}")


def scf_once(mess, mol, tau, conv_tol, max_iter=100, verbose=True, prec=0, jk_mode=0):
    B = mess.basis_from_molecule(mol)
    st = mess.mess_scf_create(B, schwarz_tol=tau, conv_tol=conv_tol, diis_size=8, prec=prec, jk_mode=jk_mode)
    e, it, conv = 0.0, 0, False
    for it in range(1, max_iter + 1):
        e, de, resid, conv = mess.mess_scf_step(st)
        if verbose:
            log(f"  iteration {it}: E={e:.10f} dE={de:.2e} resid={resid:.2e}")
        if conv:
            break
    st.close()
    B.close()
    return e, it, conv


def cpu_baseline(mol, target_seconds):
    """Oracle ERI throughput on a uniform random sample of unique shell quartets."""
    from oracle import core
    ns = mol.n_shells
    pairs = [(a, b) for a in range(ns) for b in range(a + 1)]
    rng = np.random.Generator(np.random.PCG64(12345))

    def sample(n):
        out = []
        while len(out) < n:
            i, j = rng.integers(0, len(pairs), 2)
            if j > i:
                i, j = j, i
            out.append(pairs[i] + pairs[j])
        return np.array(out, dtype=np.int32)

    core.lib()
    n = 5000
    t = time.perf_counter()
    core.eri_quartet_list(mol, sample(n))
    dt = time.perf_counter() - t
    n2 = int(max(5000, min(5000000, n * target_seconds / max(dt, 1e-3))))
    q = sample(n2)
    t = time.perf_counter()
    core.eri_quartet_list(mol, q)
    dt = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n2 / dt, "unit": "shell quartets/s", "cores": threads, "kind": "oracle",
            "sample": f"{n2} unique shell quartets of {mol.name} drawn uniformly (unscreened), "
                      f"FP64 McMurchie-Davidson oracle, {dt:.1f} s"}


def fp32_jk_error(mess, mol, a, torch):
    """max |dJ|, max |dK| of one FP32 build at the oracle's converged density
    D* against the oracle's J(D*), K(D*) (stored golden of this workload)."""
    path = os.path.join(ROOT, "tests", "golden", f"{mol.name.replace('/', '_')}_jk.npz")
    if not os.path.exists(path):
        return {}
    g = np.load(path)
    N = mol.n_bf
    iu = np.triu_indices(N)

    def full(v):
        M = np.zeros((N, N))
        M[iu] = v
        return M + np.triu(M, 1).T
    Dst, Jo, Ko = full(g["dstar_D"]), full(g["dstar_J"]), full(g["dstar_K"])
    B = mess.basis_from_molecule(mol)
    D = torch.tensor(Dst, dtype=torch.float64, device="cuda")
    J = torch.zeros(N, N, dtype=torch.float64, device="cuda")
    K = torch.zeros_like(J)
    mess.mess_jk(B, D, J, K, prec=mess.MESS_FP32, schwarz_tol=a.tau)
    torch.cuda.synchronize()
    dJ = float(np.max(np.abs(J.cpu().numpy() - Jo)))
    dK = float(np.max(np.abs(K.cpu().numpy() - Ko)))
    B.close()
    return {"max_abs_dJ_at_converged_density": dJ, "max_abs_dK_at_converged_density": dK,
            "max_abs_J": float(np.max(np.abs(Jo))), "max_abs_K": float(np.max(np.abs(Ko)))}


def recorded_traffic(class_name):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-scaled), or None when it
    covers another class or its kernel sources have changed since."""
    import hashlib
    slug = class_name.strip("()").replace("|", "_")
    path = os.path.join(ROOT, "profiles", f"hbm_counters_{slug}_water60.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("class") != class_name:
        return None
    h = hashlib.sha256()
    for src in d["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return d["hbm_bytes_per_launch"] if h.hexdigest() == d["sources_sha256"] else None


FORM_NAMES = {1: "lane", 2: "rows", 3: "plane", 4: "coop", 5: "wave", 6: "fp64"}


def autotune_block(mess, mol, a, torch):
    """Kernel form per class chosen by the library's autotuner on this
    molecule (FP64 and FP32 arithmetic), before any timed work."""
    from mess_inputs import generators as G
    B = mess.basis_from_molecule(mol)
    D = torch.tensor(G.symmetric_density(mol.n_bf, 3), dtype=torch.float64, device="cuda")
    out = {}
    for prec, name in ((mess.MESS_FP64, "fp64"), (mess.MESS_FP32, "fp32")):
        forms, ms = mess.mess_autotune(B, D, schwarz_tol=a.tau, reps=2, prec=prec)
        out[name] = {CLASS_NAMES[c]: {"form": FORM_NAMES.get(int(forms[c]), str(int(forms[c]))),
                                      "ms": {FORM_NAMES[f]: round(float(ms[c, f]), 3)
                                             for f in FORM_NAMES if ms[c, f] >= 0}}
                     for c in range(21)}
    B.close()
    log("autotuned forms (fp64): " + ", ".join(f"{k} {v['form']}" for k, v in out["fp64"].items()))
    return out


def lda_block(mess, mol, a, torch):
    """LDA exchange on the same molecule: V_x builds timed with HIP events
    (grid and basis values built beforehand), then one LDA SCF."""
    B = mess.basis_from_molecule(mol)
    n = mess.mess_grid(B)
    N = mol.n_bf
    D = torch.eye(N, dtype=torch.float64, device="cuda") * (2.0 * (mol.n_electrons // 2) / N)
    Vx = torch.zeros(N, N, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    mess.mess_lda_x(B, D, Vx)  # builds grid and basis values
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    reps = 5
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        mess.mess_lda_x(B, D, Vx, None)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    flops = 4.0 * N * N * n  # rho: 2 N^2 per point; V_x: 2 N^2 per point
    tf = flops / (ms * 1e-3) / 1e12
    B.close()
    B = mess.basis_from_molecule(mol)
    t1 = time.perf_counter()
    st = mess.mess_scf_create(B, schwarz_tol=a.tau, conv_tol=a.conv, diis_size=8, xc=mess.MESS_XC_LDA_X)
    e, it, conv = 0.0, 0, False
    for it in range(1, 101):
        e, de, resid, conv = mess.mess_scf_step(st)
        if conv:
            break
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st.close()
    return {"grid_points": n, "grid_and_basis_values_s": build_s, "vx_ms_per_build": ms,
            "vx_alg_tflops": tf, "vx_frac_of_fp64_peak": tf / FP64_VALU_PEAK_TFLOPS,
            "scf_s": t2 - t1, "scf_iterations": it, "scf_converged": bool(conv), "energy_hartree": e}


def cpu_baseline_batch_check(mols, energies, converged, count=8, max_nbf=40):
    """CPU-baseline leg: |E - E_oracle| on a sample of converged molecules
    small enough for the dense oracle (the smallest ones): (checked, within
    1e-6 Ha, max |dE|)."""
    from oracle import scf as oscf
    idx = [m for m in sorted(range(len(mols)), key=lambda m: mols[m].n_bf)
           if converged[m] and mols[m].n_bf <= max_nbf][:count]
    worst, ok = 0.0, 0
    for m in idx:
        ref = oscf.RHF(mols[m], jk="dense", conv_tol=1e-10, max_iter=200).run()
        d = float(abs(energies[m] - ref["energy"]))
        worst = max(worst, d)
        ok += int(d < 1e-6)
    return len(idx), ok, worst


def batch_block(mess, a, torch, jk_mode=0, prec=0):
    """Batched SCF over many small molecules (seeds 1000...), one HIP graph
    per step, a fixed number of steps; jk_mode 1 stores the integral blocks
    at set-up and streams them in every step; prec 1 is the mixed-precision
    batch.  Direct-J/K batches first let the autotuner choose the kernel
    forms on the batch (unless --no-tune).  Returns the figures and what the CPU-baseline leg checks
    (converged molecules count toward molecules/s in proportion to the share
    of an oracle-checked sample within 1e-6 Ha)."""
    from mess_inputs import generators as G
    mols = G.batch_of_molecules(a.batch_molecules)
    t0 = time.perf_counter()
    B = mess.mess_batch_create(mols)
    bs = mess.mess_batch_scf_create(B, schwarz_tol=a.tau, conv_tol=a.conv, diis_size=8, use_graph=True,
                                    jk_mode=jk_mode, prec=prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tuned = None
    if not a.no_tune and jk_mode == 0:
        # the library's autotuner on the batch itself (its best forms differ
        # from the 60-atom cluster's for a few classes), in the arithmetic the
        # steps use; a one-time choice, kept out of the set-up and rate figures
        D = torch.zeros(B.packed, dtype=torch.float64, device="cuda")
        mess.mess_batch_scf_density(bs, D)
        tuned = {}
        for p, name in ((mess.MESS_FP64, "fp64"), (mess.MESS_FP32, "fp32")):
            if p == mess.MESS_FP32 and prec != mess.MESS_FP32:
                continue
            forms, _ = mess.mess_autotune(B, D, schwarz_tol=a.tau, reps=2, prec=p)
            tuned[name] = {CLASS_NAMES[c]: FORM_NAMES.get(int(forms[c]), str(int(forms[c]))) for c in range(21)}
        torch.cuda.synchronize()
        tuned["s"] = time.perf_counter() - t1
        t0 += tuned["s"]
        t1 = time.perf_counter()
    if a.mark_steps > 0:
        time.sleep(a.mark_steps)
        t0 += time.perf_counter() - t1  # the idle mark is in no figure
        t1 = time.perf_counter()
    conv_hist = []
    for k in range(a.batch_steps):
        mess.mess_batch_scf_step(bs)
        st = mess.mess_batch_scf_status(bs)
        conv_hist.append(st["n_converged"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    q = sum(mess.mess_work_stats(B, a.tau, c)[0] for c in range(21))
    stages = mess.mess_batch_scf_guard(bs)
    bs.close()
    out = {"molecules": len(mols), "n_bf_total": int(B.nbf), "packed_doubles": int(B.packed),
           "shell_quartets_per_step": q, "setup_s": t1 - t0, "steps": a.batch_steps,
           "ms_per_step": (t2 - t1) / a.batch_steps * 1e3, "converged_after_steps": conv_hist,
           "guard_stage_counts": [int(np.sum(stages == k)) for k in range(4)],
           "converged_molecules_per_s_unchecked": conv_hist[-1] / (t2 - t0),
           "converged_molecules_per_s": None,
           "shell_quartets_per_s": q * a.batch_steps / (t2 - t1)}
    if tuned is not None:
        out["autotune"] = tuned
    # kept for the oracle check of the CPU-baseline leg
    check = (mols, st["energy"].copy(), st["converged"].copy(), conv_hist[-1], t2 - t0)
    return out, check


def gate_batch(out, check, verdict):
    """Batch molecules/s counting converged molecules in proportion to the
    share of the oracle-checked sample within 1e-6 Ha."""
    nchk, nok, worst = verdict
    out.update({"oracle_checked": nchk, "oracle_within_1e-6": nok, "oracle_max_abs_de": worst,
                "converged_molecules_per_s": check[3] * (nok / nchk if nchk else 0.0) / check[4]})


def dmin_block(mess, a, torch):
    """Direct minimisation (QR + Adam, lr 0.1) of the 6-atom s/p molecule:
    time per step and steps until the energy is within 1e-6 Ha of the SCF's."""
    from mess_inputs import generators as G
    mol = G.random_small_molecule(1)
    B = mess.basis_from_molecule(mol)
    sc = mess.mess_scf_create(B, schwarz_tol=a.tau, conv_tol=1e-11, diis_size=8)
    for _ in range(100):
        e_scf, de, r, c = mess.mess_scf_step(sc)
        if c:
            break
    st = mess.mess_scf_create(B, schwarz_tol=a.tau, conv_tol=0.0, diis_size=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reached, n = None, 0
    for n in range(1, 801):
        e, g = mess.mess_dmin_step(st, lr=0.1)
        if reached is None and abs(e - e_scf) < 1e-6:
            reached = n
            break
    t1 = time.perf_counter()
    return {"workload": mol.name, "n_bf": mol.n_bf, "steps_to_1e-6": reached, "ms_per_step": (t1 - t0) / n * 1e3,
            "energy_hartree": e, "scf_energy_hartree": e_scf}


def scan_block(mess, a, torch):
    """Conformer scan: 64 geometries of a 19-atom molecule (one bond
    stretched) as one batch; SCF of every conformer to |dE| < conv."""
    from mess_inputs import generators as G
    base = G.batched_molecule(1001)
    d = base.xyz[1] - base.xyz[0]
    mols = G.conformer_scan(base, 1, d, np.linspace(-0.3, 1.5, 64))
    t0 = time.perf_counter()
    B = mess.mess_batch_create(mols)
    bs = mess.mess_batch_scf_create(B, schwarz_tol=a.tau, conv_tol=a.conv, diis_size=8, use_graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps = 0
    for steps in range(1, 61):
        mess.mess_batch_scf_step(bs)
        st = mess.mess_batch_scf_status(bs)
        if st["n_converged"] == len(mols):
            break
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bs.close()
    return {"conformers": len(mols), "n_bf_each": base.n_bf, "steps": steps, "converged": st["n_converged"],
            "setup_s": t1 - t0, "scf_s": t2 - t1, "conformers_per_s": st["n_converged"] / (t2 - t0),
            "energy_min_hartree": float(np.min(st["energy"])), "energy_max_hartree": float(np.max(st["energy"]))}


def small_block(mess, a, torch, n_seeds=64):
    """The 6-atom H/C/O s/p molecules (about 30 functions): latency of the
    full ERI tensor and of one direct J/K build (3 warm-ups, median of 10,
    seed 0), the 20-iteration plain Roothaan SCF (no DIIS, no guard) of every
    seed, and the analytic nuclear gradient at seed 0's converged SCF.  Returns the figures and what the CPU-baseline leg checks."""
    from mess_inputs import generators as G

    def median_ms(fn, reps=10, warm=3):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return float(np.median(ts))

    def roothaan20(B):
        st = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=0.0, diis_size=0, guard=False)
        es = [mess.mess_scf_step(st)[0] for _ in range(20)]
        st.close()
        return es

    mol = G.random_small_molecule(0)
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    n_sh = mol.n_shells
    n_pairs = n_sh * (n_sh + 1) // 2
    eri = torch.zeros(N, N, N, N, dtype=torch.float64, device="cuda")
    D = torch.tensor(G.symmetric_density(N, 5), dtype=torch.float64, device="cuda")
    J, K = torch.zeros(N, N, dtype=torch.float64, device="cuda"), torch.zeros_like(D)
    eri_ms = median_ms(lambda: mess.mess_eri(B, eri, schwarz_tol=0.0))
    jk_ms = median_ms(lambda: mess.mess_jk(B, D, J, K, schwarz_tol=0.0))
    scf_ms = median_ms(lambda: roothaan20(B), reps=5, warm=1)
    es = roothaan20(B)
    # analytic nuclear gradient at the converged (DIIS) SCF
    sc = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=1e-10, diis_size=8)
    for _ in range(100):
        if mess.mess_scf_step(sc)[3]:
            break
    grad_ms = median_ms(lambda: mess.mess_scf_gradient(sc), reps=5, warm=1)
    gnorm = float(np.abs(mess.mess_scf_gradient(sc)).max())
    sc.close()
    torch.cuda.synchronize()
    check = (mol, eri.cpu().numpy(), J.cpu().numpy(), K.cpu().numpy(), es)
    B.close()
    # every seed: 20 Roothaan iterations
    t = time.perf_counter()
    for seed in range(n_seeds):
        Bs = mess.basis_from_molecule(G.random_small_molecule(seed))
        roothaan20(Bs)
        Bs.close()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t
    return {"workload": "hco6_sp", "seed": 0, "n_bf": N, "n_shells": n_sh,
            "unique_shell_quartets": n_pairs * (n_pairs + 1) // 2,
            "eri_tensor_ms": eri_ms, "eri_per_s": N ** 4 / (eri_ms * 1e-3),
            "jk_ms": jk_ms, "scf20_ms": scf_ms, "energy_after_20_hartree": es[-1],
            "gradient_ms": grad_ms, "max_abs_gradient": gnorm,
            "seeds": n_seeds, "scf20_all_seeds_s": t_all, "scf20_molecules_per_s": n_seeds / t_all}, check


def dense_block(mess, a, torch, nd=64):
    """J and K of 64 densities from the dense ERI tensor of a 105-function
    molecule (batched seed 1000; tensor 970 MB in FP64), matrix-core and
    vector forms, FP64 and FP32: time per J+K pair (median of 5 after 2
    warm-ups, stream events) and algorithmic TFLOP/s (2 n^4 flops per
    density for each of J and K) against the dense peaks (FP64 78.6, FP32
    matrix cores 157.3, FP32 vector FMAs without packed math 78.6)."""
    from mess_inputs import generators as G
    mol = G.batched_molecule(1000)
    B = mess.basis_from_molecule(mol)
    n = B.nbf
    out = {"workload": "mol3to20_spd/1000", "n_bf": n, "densities": nd}
    rng = np.random.Generator(np.random.PCG64(3))
    for prec, dt, name in ((mess.MESS_FP64, torch.float64, "fp64"), (mess.MESS_FP32, torch.float32, "fp32")):
        eri = torch.zeros(n, n, n, n, dtype=torch.float64, device="cuda")
        mess.mess_eri(B, eri, prec=prec, schwarz_tol=0.0)  # dense tensors are written as doubles
        eri = eri.to(dt)
        A = rng.normal(size=(nd, n, n)) / n
        D = torch.tensor(A + A.transpose(0, 2, 1), dtype=dt, device="cuda")
        J, K = torch.zeros_like(D), torch.zeros_like(D)
        res = {}
        for form, fname in ((mess.MESS_DENSE_MFMA, "mfma"), (mess.MESS_DENSE_VALU, "valu")):
            for _ in range(2):
                mess.mess_jk_dense(eri, n, D, J, K, prec=prec, form=form)
            ts = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mess.mess_jk_dense(eri, n, D, J, K, prec=prec, form=form)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            tf = 2 * 2.0 * n ** 4 * nd / (ms * 1e-3) / 1e12
            peak = 157.3 if (name == "fp32" and fname == "mfma") else 78.6
            res[fname] = {"ms": ms, "alg_tflops": tf, "frac": tf / peak}
        out[name] = res
        del eri
    B.close()
    return out


def cpu_baseline_small(check):
    """CPU-baseline leg for the 6-atom molecule: the oracle's times (dense
    ERI tensor, one J/K contraction, 20 Roothaan iterations; one process) and
    the GPU results' differences from its values."""
    from mess_inputs import generators as G
    from oracle import core
    from oracle import scf as oscf
    mol, eri, J, K, es = check
    t = time.perf_counter()
    eri_o = core.eri_dense(mol)
    t_eri_o = time.perf_counter() - t
    t = time.perf_counter()
    Jo, Ko = core.jk_from_dense(eri_o, G.symmetric_density(mol.n_bf, 5))
    t_jk_o = time.perf_counter() - t
    t = time.perf_counter()
    ro = oscf.RHF(mol, jk="dense", diis=False, fixed_iters=20, guard=False).run()
    t_scf_o = time.perf_counter() - t
    return {"eri_tensor_s": t_eri_o, "jk_s": t_jk_o, "scf20_s": t_scf_o, "kind": "oracle",
            "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "max_abs_d_eri": float(np.max(np.abs(eri - eri_o))), "max_abs_d_j": float(np.max(np.abs(J - Jo))),
            "max_abs_d_k": float(np.max(np.abs(K - Ko))),
            "delta_e_after_20_hartree": es[-1] - ro["energies"][-1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="water60_spd")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tau", type=float, default=1e-10)
    ap.add_argument("--conv", type=float, default=1e-8)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-stored", action="store_true", help="skip the stored-J/K comparison")
    ap.add_argument("--no-lda", action="store_true", help="skip the LDA-exchange measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the 1024-molecule batched SCF")
    ap.add_argument("--batch-molecules", type=int, default=1024)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in kernel forms")
    ap.add_argument("--no-dmin", action="store_true", help="skip the direct-minimisation measurement")
    ap.add_argument("--no-scan", action="store_true", help="skip the conformer scan")
    ap.add_argument("--no-oracle-check", action="store_true", help="skip the oracle check of batch energies")
    ap.add_argument("--no-small", action="store_true", help="skip the 6-atom latency measurements")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-tensor J/K contraction")
    ap.add_argument("--mark-steps", type=float, default=0.0,
                    help="idle seconds before the timed steps of the batch blocks, so that a kernel trace shows "
                         "where they begin (outside the timed region)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU split of the "
              "shell-quartet lists is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_03121_amd import mess
    torch.cuda.init()
    mol = make_workload(a.workload, a.seed)
    log(f"workload {mol.name}: {mol.n_atoms} atoms, {mol.n_shells} shells, {mol.n_bf} functions")
    tune = None if a.no_tune else autotune_block(mess, mol, a, torch)
    for w in range(a.warmup):
        e, it, conv = scf_once(mess, mol, a.tau, a.conv)
        log(f"warmup {w}: E={e:.10f} iterations={it} converged={conv}")

    torch.cuda.synchronize()
    mess.mess_prof_enable(True)
    t0 = time.perf_counter()
    results = []
    for k in range(a.steps):
        results.append(scf_once(mess, mol, a.tau, a.conv))
        log(f"step {k}: E={results[-1][0]:.10f} iterations={results[-1][1]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    tot = mess.mess_prof_read(-1)
    per = {}
    for c in range(21):
        r = mess.mess_prof_read(c)
        if r["launches"]:
            per[c] = r
    mess.mess_prof_enable(False)

    dom = max(per, key=lambda c: per[c]["ms"])
    d = per[dom]
    achieved = d["alg_flops"] / (d["ms"] * 1e-3) / 1e12
    eri_tf = tot["alg_flops"] / (tot["ms"] * 1e-3) / 1e12
    value = tot["quartets"] / elapsed
    energies = [r[0] for r in results]
    line = {
        "metric": "shell-quartet ERIs/s + J/K GB/s; SCF molecules/s vs plain FP64 at |ΔE|<1e-6 Ha",
        "value": value,
        "unit": "shell quartets/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "seed": a.seed, "n_atoms": mol.n_atoms, "n_bf": mol.n_bf,
                   "schwarz_tol": a.tau, "conv_tol": a.conv, "jk": "direct", "diis": 8},
        "molecules_per_s": a.steps / elapsed,
        "scf_iterations": results[-1][1],
        "energy_hartree": energies[-1],
        "energy_spread_hartree": float(np.max(energies) - np.min(energies)),
        "jk_gbps": None,
        "primitive_quartets_per_s": tot["prim_quartets"] / elapsed,
        "eri_kernels": {"ms": tot["ms"], "alg_tflops": eri_tf, "frac_of_fp64_peak": eri_tf / FP64_VALU_PEAK_TFLOPS,
                        "share_of_step": tot["ms"] * 1e-3 / elapsed},
        "per_class": {CLASS_NAMES[c]: {"ms": round(per[c]["ms"], 3), "quartets": per[c]["quartets"],
                                       "prim_quartets": per[c]["prim_quartets"],
                                       "tflops": round(per[c]["alg_flops"] / (per[c]["ms"] * 1e-3) / 1e12, 3)}
                      for c in sorted(per)},
        "roofline": {"kernel": f"ERI/JK class {CLASS_NAMES[dom]}", "bound": "alu",
                     "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": recorded_traffic(CLASS_NAMES[dom])},
        "cpu_baseline": None,
    }
    if tune is not None:
        line["autotune"] = tune
    golden = os.path.join(ROOT, "tests", "golden", f"{mol.name.replace('/', '_')}_rhf.json")
    if os.path.exists(golden):
        ref = json.load(open(golden))["energy"]
        line["delta_e_vs_oracle_hartree"] = energies[-1] - ref
    if not a.no_fp32:
        # same molecule, mixed precision, timed like the FP64 run (class
        # events on), per-class kernel times in both arithmetics
        scf_once(mess, mol, a.tau, a.conv, verbose=False, prec=mess.MESS_FP32)
        torch.cuda.synchronize()
        mess.mess_prof_enable(True)
        t2 = time.perf_counter()
        r32 = [scf_once(mess, mol, a.tau, a.conv, verbose=False, prec=mess.MESS_FP32) for _ in range(a.steps)]
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        pc32 = {}
        for c in range(21):
            r64, r32c = mess.mess_prof_read(c), mess.mess_prof_read(64 + c)
            pc32[CLASS_NAMES[c]] = {
                "fp32_ms_per_launch": round(r32c["ms"] / r32c["launches"], 4) if r32c["launches"] else None,
                "fp64_ms_per_launch": round(per[c]["ms"] / per[c]["launches"], 4) if c in per else None,
                "fp32_launches": r32c["launches"], "fp64_launches": r64["launches"]}
        mess.mess_prof_enable(False)
        fp32 = {"ms_per_step": (t3 - t2) / a.steps * 1e3, "molecules_per_s": a.steps / (t3 - t2),
                "scf_iterations": r32[-1][1], "energy_hartree": r32[-1][0],
                "delta_e_vs_fp64_hartree": r32[-1][0] - energies[-1], "per_class": pc32}
        fp32["speedup_vs_fp64"] = fp32["molecules_per_s"] / line["molecules_per_s"]
        if "delta_e_vs_oracle_hartree" in line:
            fp32["delta_e_vs_oracle_hartree"] = r32[-1][0] - ref
        fp32.update(fp32_jk_error(mess, mol, a, torch))
        line["fp32_mixed"] = fp32
        log(f"fp32: {dict((k, v) for k, v in fp32.items() if k != 'per_class')}")
    if not a.no_stored:
        # same molecule, stored J/K: blocks computed once per SCF (first
        # Fock build), streamed from HBM by the later builds
        scf_once(mess, mol, a.tau, a.conv, verbose=False, jk_mode=mess.MESS_JK_STORED)
        torch.cuda.synchronize()
        mess.mess_prof_enable(True)
        t4 = time.perf_counter()
        rst = [scf_once(mess, mol, a.tau, a.conv, verbose=False, jk_mode=mess.MESS_JK_STORED)
               for _ in range(a.steps)]
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        sb, sms = 0.0, 0.0
        spc = {}
        nb = max(1, a.steps * (rst[-1][1] - 1))
        for c in range(21):
            r = mess.mess_prof_read(32 + c)
            sb += r["alg_flops"]
            sms += r["ms"]
            if r["launches"] and r["ms"] > 0:
                spc[CLASS_NAMES[c]] = {"ms_per_build": round(r["ms"] / nb, 3),
                                       "gbps": round(r["alg_flops"] / (r["ms"] * 1e-3) / 1e9, 1)}
        mess.mess_prof_enable(False)
        stored = {"ms_per_step": (t5 - t4) / a.steps * 1e3, "molecules_per_s": a.steps / (t5 - t4),
                  "scf_iterations": rst[-1][1], "energy_hartree": rst[-1][0],
                  "delta_e_vs_direct_hartree": rst[-1][0] - energies[-1],
                  "jk_stream_bytes_per_build": sb / max(1, a.steps * (rst[-1][1] - 1)),
                  "jk_stream_ms_per_build": sms / max(1, a.steps * (rst[-1][1] - 1)),
                  "jk_gbps": sb / (sms * 1e-3) / 1e9 if sms > 0 else None,
                  "speedup_vs_direct": (a.steps / (t5 - t4)) / line["molecules_per_s"],
                  "per_class_stream": spc}
        line["stored_jk"] = stored
        line["jk_gbps"] = stored["jk_gbps"]
        log(f"stored: {stored}")
    checks = {}
    if not a.no_small:
        line["small_molecule"], checks["small_molecule"] = small_block(mess, a, torch)
        log(f"small molecule: {line['small_molecule']}")
    if not a.no_dense:
        line["dense_jk"] = dense_block(mess, a, torch)
        log(f"dense jk: {line['dense_jk']}")
    if not a.no_lda:
        line["lda"] = lda_block(mess, mol, a, torch)
        log(f"lda: {line['lda']}")
    if not a.no_batch:
        line["batch"], checks["batch"] = batch_block(mess, a, torch)
        log(f"batch: {line['batch']}")
        if not a.no_fp32:
            line["batch_fp32_mixed"], checks["batch_fp32_mixed"] = batch_block(mess, a, torch, prec=mess.MESS_FP32)
            log(f"batch (mixed precision): {line['batch_fp32_mixed']}")
        if not a.no_stored:
            line["batch_stored_jk"], checks["batch_stored_jk"] = batch_block(mess, a, torch,
                                                                             jk_mode=mess.MESS_JK_STORED)
            log(f"batch (stored J/K): {line['batch_stored_jk']}")
    if not a.no_scan:
        line["conformer_scan"] = scan_block(mess, a, torch)
        log(f"scan: {line['conformer_scan']}")
    if not a.no_dmin:
        line["direct_minimisation"] = dmin_block(mess, a, torch)
        log(f"dmin: {line['direct_minimisation']}")
    if not a.no_cpu_baseline:
        # the CPU-baseline leg: the oracle timed on a quartet sample, and the
        # oracle's values that the results above are checked against
        log("timing the CPU oracle on a quartet sample")
        cb = cpu_baseline(mol, a.cpu_seconds)
        if "small_molecule" in checks:
            cb["small_molecule"] = cpu_baseline_small(checks["small_molecule"])
            line["small_molecule"]["oracle"] = cb["small_molecule"]
        for key in ("batch", "batch_fp32_mixed", "batch_stored_jk"):
            if key in checks and not a.no_oracle_check:
                mols, e, c, nconv, dt = checks[key]
                gate_batch(line[key], checks[key], cpu_baseline_batch_check(mols, e, c))
        line["cpu_baseline"] = cb
    print(json.dumps(line, default=lambda o: o.item() if hasattr(o, "item") else str(o)), flush=True)


if __name__ == "__main__":
    main()
