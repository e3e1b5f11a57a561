"""Throughput of the F12 integral path on one MI355X.

One step evaluates one batch of the 20-atom molecule's unique shell quartets
(seed 5070; per atom s, s, p, p, d, f shells with 1-6 primitives, exponents
log-uniform in [0.05, 50]; factor set P1) for every class I2-I6: radial
derivatives of the basic integrals, Hermite integrals, E.R.E contraction,
contracted blocks written to an HBM ring buffer.  The quartet list of each
class is split into --batches batches: batch b takes slice (b + g) mod
batches of the g-th (l_a, l_b, l_c, l_d) group (groups are ordered by
decreasing primitive count), so each step mixes heavy and light slices,
successive steps cover different quartets and --batches steps cover the
whole job.  Inputs are resident in HBM before the
timed region.

Prints one JSON line: contracted quartets/s over the timed steps (all
classes), per-class rates, a roofline entry for the contraction kernel with
the largest share of the time (algorithmic FP64 flops per launch over its
launch time, both measured here with HIP events on the launch stream), and
the CPU oracle's rate on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (256 CUs x 2.4 GHz x 128 flop/clk)
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
CLASSES = (2, 3, 4, 5, 6)
METRIC = "contracted shell-quartets/s per F12 class at ≤1e-12 rel err; % FP64 peak"

# HBM traffic per launch of the contraction and radial-derivative kernels,
# from two rocprofv3 --pmc passes over this script's default run (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch, averaged over the launches of the timed
# steps), each counter scaled by what it reads for a plain 1 GiB device copy
# (--copy-probe): FETCH_SIZE reads half the bytes fetched, WRITE_SIZE all of
# them.  The figures hold only for the kernel sources they were taken on: the
# SHA-1 covers those files, and traffic is reported as null once they differ.
# Summary and commands: profiles/contraction_hbm_traffic.md.
KERNEL_SOURCES = ["f12_big.h", "f12_common.h", "f12_launch.h", "f12_internal.h", "f12_kernels.hip",
                  "f12_dd.h", "f12_big_unit.hip"]
TRAFFIC_RECORD = {
    "sources_sha1": "f853387ce201a7e7018054ab771dbd2dbc23c7cb",
    "fetch_scale": 1048576 / 524299.5,
    "write_scale": 1.0,
    "contraction_bytes_per_launch": 6.47169e+07 + 1.37969e+08,
    "aux_bytes_per_launch": 3.38034e+08 + 5.82893e+08,
    # FP64 flops issued per launch, 64 lanes x (2 SQ_INSTS_VALU_FMA_F64 + SQ_INSTS_VALU_MUL_F64 +
    # SQ_INSTS_VALU_ADD_F64), from one more --pmc pass (profiles/contraction_fp64_counters.md);
    # an upper bound, since lanes masked off are counted too
    "contraction_hw_fp64_flops_per_launch": 3.128e+10,
    "aux_hw_fp64_flops_per_launch": 8.651e+09,
}


def kernel_sources_sha1():
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1412_5070_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# algorithmic work per launch (FP64 flops the method must perform)
# ---------------------------------------------------------------------------
def _hs3(L):
    return (L + 1) * (L + 2) * (L + 3) // 6 if L >= 0 else 0


def _nc(l):
    return (l + 1) * (l + 2) // 2


def _carts(l):
    return [(i, k, l - i - k) for i in range(l, -1, -1) for k in range(l - i, -1, -1)]


def _ket_fmas(Lab, lc, Lcd):
    """FMAs of the three one-dimensional ket passes for one primitive quartet."""
    z = 0
    for v in range(Lab + 1):
        for fz in range(Lcd + 1):
            m = Lab - v + Lcd - fz
            z += (m + 1) * (m + 2) // 2 * (fz + 1)
    y = 0
    for u in range(Lab + 1):
        for v in range(Lab + 1 - u):
            for fy in range(Lcd + 1):
                for fz in range(Lcd + 1 - fy):
                    y += (Lab - u - v + Lcd - fy - fz + 1) * (fy + 1)
    x = 0
    for t in range(Lab + 1):
        for u in range(Lab + 1 - t):
            for v in range(Lab + 1 - t - u):
                for f in range(lc, Lcd + 1):
                    for (fx, _, _) in _carts(f):
                        x += fx + 1
    return z + y + x


def _bra_fmas(la, Lab, nf):
    """FMAs of a factorised bra transform for one bra primitive."""
    x = sum(ex + 1 for ex in range(Lab + 1) for u in range(Lab + 1) for v in range(Lab + 1 - u)
            if u + v <= Lab - ex)
    y = sum(ey + 1 for ex in range(Lab + 1) for ey in range(Lab + 1 - ex) for v in range(Lab + 1 - ex - ey))
    z = sum(ez + 1 for e in range(la, Lab + 1) for (_, _, ez) in _carts(e))
    return (x + y + z) * nf


def _hrr_fmas(la, lb, lc, ld):
    n = 0
    for (dx, dy, dz) in _carts(ld):
        n += (dx + 1) * (dy + 1) * (dz + 1)
    return n * _nc(la) * _nc(lb) * _nc(lc)


def contraction_flops(la, lb, lc, ld, i5, n_prim, n_bra_prim, n_quartets):
    """Algorithmic FP64 flops of one contraction launch: R recursion, ket
    passes, bra transform, transfer to (cd); I5 runs four components."""
    Lab, Lcd = la + lb, lc + ld
    L = Lab + Lcd + (2 if i5 else 0)
    ncomp = 4 if i5 else 1
    nf = _hs3(Lcd) - _hs3(lc - 1)
    r = sum(_hs3(L - n) for n in range(L + 1))
    per_prim = 2 * r + ncomp * 2 * _ket_fmas(Lab, lc, Lcd) + (2 * _hs3(Lab + Lcd) if i5 else 0)
    per_bra = ncomp * 2 * _bra_fmas(la, Lab, nf)
    return per_prim * n_prim + per_bra * n_bra_prim + 2 * _hrr_fmas(la, lb, lc, ld) * n_quartets


def e_nonzero_fraction(la, lb):
    """Fraction of the dense bra tile E^ab_{tuv} (n_a n_b x H(l_a + l_b)) that is
    nonzero: component pair (a, b) reaches t <= a_x + b_x, u <= a_y + b_y,
    v <= a_z + b_z."""
    nz = 0
    for (ax, ay, az) in _carts(la):
        for (bx, by, bz) in _carts(lb):
            nz += (ax + bx + 1) * (ay + by + 1) * (az + bz + 1)
    return nz / (_nc(la) * _nc(lb) * _hs3(la + lb))


def method_flops(la, lb, lc, ld, i5, n_prim, n_bra_prim):
    """Algorithmic FP64 flops of one contraction launch by the method's own
    per-unit count (what the E.R.E route must compute, not the dense 6-D work
    it avoids):
      per primitive quartet: 3 C(L+4, 4) for the Hermite integrals R_tuv of
        every order n (L = l_a+l_b+l_c+l_d, +2 for I5), plus the ket transform
        2 H(L_ab) H(L_cd) n_c n_d (H(L) = (L+1)(L+2)(L+3)/6 Hermite functions);
      per bra primitive pair (after the ket primitives are summed): the bra
        transform 2 n_a n_b H(L_ab) n_c n_d times the nonzero fraction of E^ab;
      I5: four components (the Laplacian shift and three gradients), so 4x the
        ket and bra terms, with R at L + 2 (Eq. (I5byI3_))."""
    Lab, Lcd = la + lb, lc + ld
    L = Lab + Lcd + (2 if i5 else 0)
    ncomp = 4 if i5 else 1
    ncd = _nc(lc) * _nc(ld)
    per_prim = 3 * math.comb(L + 4, 4) + ncomp * 2 * _hs3(Lab) * _hs3(Lcd) * ncd
    per_bra = ncomp * 2 * _nc(la) * _nc(lb) * _hs3(Lab) * ncd * e_nonzero_fraction(la, lb)
    return per_prim * n_prim + per_bra * n_bra_prim


def kernel_chains(terms):
    """Chains of the kernel's term table (equal b, g and alpha mod 1): their
    count and, per chain, the span of integer power offsets."""
    ch = {}
    for (c, alpha, b, g) in terms:
        a0 = alpha - math.floor(alpha + 1e-9)
        if a0 < 1e-9 or a0 > 1 - 1e-9:
            a0 = 0.0
        key = (round(b, 9), round(g, 9), round(a0, 9))
        m = int(round(alpha - a0))
        lo, hi = ch.get(key, (m, m))
        ch[key] = (min(lo, m), max(hi, m))
    return [hi - lo for (lo, hi) in ch.values()]


# flops of the start of one auxiliary-function ladder: one table row read and
# its Taylor shift (16 terms, 2 flops each), plus the exponential and the
# power of gamma that scale it
AUX_START_FLOPS = 2 * 16 + 20 + 20


def aux_flops(L, spans, n_prim):
    """Algorithmic FP64 flops of the auxiliary functions and radial derivatives
    A_0..A_L of n_prim primitive quartets:
      per chain and per sign (+, -): a ladder start and (L + span) steps of
        about 6 flops;
      per sign: the recursion to the radial derivatives, about
        2 x 4 flops x (L+1)(L+2)(2L+3)/6 entries."""
    per = 0
    for span in spans:
        per += 2 * (AUX_START_FLOPS + 6 * (L + span))
    per += 2 * 2 * 4 * (L + 1) * (L + 2) * (2 * L + 3) // 6
    return per * n_prim


def kernel_name(la, lb, lc, ld, i5):
    """The big_kernel instantiation family of a shell-quartet shape."""
    return "big_kernel, l_a+l_b=%d, l_c+l_d=%d%s" % (la + lb, lc + ld, ", I5" if i5 else "")


# ---------------------------------------------------------------------------
# CPU oracle on a bounded sample
# ---------------------------------------------------------------------------
CPU_BINS = ((1, 4), (5, 16), (17, 64))


def _cpu_worker(job):
    """One worker of the CPU baseline: evaluate quartets of one stratum (class,
    primitive-count bin) drawn uniformly from it with the oracle until the
    time budget is used (at least one); returns (stratum, quartets, seconds)."""
    stratum, seed, budget_s, cand = job
    cls = stratum[0]
    from oracle import integrals
    from synth import FACTOR_SETS, config_plain
    P1 = FACTOR_SETS["P1"]
    _, shells = config_plain()
    rng = np.random.default_rng(seed)
    used, n = 0.0, 0
    while used < budget_s or n < 1:
        q = cand[int(rng.integers(len(cand)))]
        sh = [shells[i].as_dict() for i in q]
        t0 = time.perf_counter()
        integrals.contracted(cls, *sh, P1, P1)
        used += time.perf_counter() - t0
        n += 1
    return stratum, n, used


def cpu_baseline(work, ks, budget_s=20.0, seed=7):
    """Oracle rate on the host cores over a stratified sample of the workload:
    strata are (class, primitive-count bin) with bins of 1-4, 5-16 and 17-64
    primitive quartets; one worker process per core takes one stratum (strata
    dealt round-robin), draws quartets uniformly from it and times the oracle
    on each until its budget is used.  The mean time per quartet of the
    covered part of the workload is the stratum means weighted by the
    workload's quartet counts, t = sum_s w_s t_s / sum_s w_s, and the rate on
    C cores is C / t.  Quartets with more than 64 primitive quartets (minutes
    each in the oracle) are not sampled: the reported coverage is the share
    of the workload's quartets the strata hold.  Workers are started fresh
    (spawn) and never touch the GPU."""
    import multiprocessing as mp
    strata, total = [], 0
    for wk in work:
        quads = wk["quads_all"]
        pq = ks[quads].prod(axis=1)
        total += len(quads)
        for (lo, hi) in CPU_BINS:
            idx = np.nonzero((pq >= lo) & (pq <= hi))[0]
            if len(idx) == 0:
                continue
            rng = np.random.default_rng(seed + wk["cls"] * 10 + lo)
            pick = rng.choice(idx, size=min(512, len(idx)), replace=False)
            strata.append(((wk["cls"], lo, hi), len(idx), [tuple(int(v) for v in quads[i]) for i in pick]))
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    cores = max(1, min(16, cores, os.cpu_count() or 1))
    jobs = [(strata[w % len(strata)][0], seed + 1000 * w, budget_s, strata[w % len(strata)][2])
            for w in range(max(cores, len(strata)))]
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map_async(_cpu_worker, jobs).get(timeout=20 * budget_s + 600)
    acc = {}
    for (st, n, used) in res:
        a = acc.setdefault(st, [0, 0.0])
        a[0] += n
        a[1] += used
    wsum = sum(w for (st, w, _) in strata)
    tbar = sum(w * acc[st][1] / acc[st][0] for (st, w, _) in strata) / wsum
    per = {"I%d %d-%d" % st: {"quartets_timed": acc[st][0], "s_per_quartet": acc[st][1] / acc[st][0],
                              "workload_quartets": w} for (st, w, _) in strata}
    return {"rate": cores / tbar, "rate_one_core": 1.0 / tbar, "cores": cores, "coverage": wsum / total,
            "quartets_timed": sum(a[0] for a in acc.values()), "cpu_seconds": sum(a[1] for a in acc.values()),
            "strata": per}


def copy_probe(nbytes):
    """A fill of nbytes, then three copies of nbytes between two HBM buffers."""
    import torch
    n = nbytes // 8
    src = torch.empty(n, dtype=torch.float64, device="cuda")
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3, "fills": 1}))


def i5_vanishes(qd, shells):
    """An I5 block vanishes identically when the bra is one shell taken twice
    and either the shell is s or p (the Laplacian of each component is the
    component times one radial function), or the ket is two s shells on the
    bra's centre (the bra density difference is the divergence of
    phi_b grad phi_a - phi_a grad phi_b, the ket's potential is spherical about
    that centre, and the radial parts of the flux cancel for two components of
    one shell).  Such blocks are scored against the size of the cancelling
    terms, not against their own rounding noise."""
    a, b, c, d = (shells[int(i)] for i in qd)
    if int(qd[0]) != int(qd[1]):
        return False
    if a.l <= 1:
        return True
    same = lambda x, y: np.allclose(x.center, y.center, rtol=0.0, atol=1e-12)
    return c.l == 0 and d.l == 0 and same(a, c) and same(a, d)


def stored_sample_errors(work, shells):
    """Block errors of each class against the stored oracle values of quartets
    sampled from the 20-atom list (tests/golden/plain20.npz, written by the
    oracle), evaluated one quartet per launch through the same list.  Every
    block is scored block-relative, max |I_gpu - I_ref| / max |I_ref|; an I5
    block that vanishes identically (i5_vanishes) is scored against the largest
    bra exponent times max |I3|."""
    import torch
    from paper_1412_5070_amd import f12int
    path = os.path.join(ROOT, "tests", "golden", "plain20.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        gold = {k: z[k] for k in z.files}
    res = {}
    for wk in work:
        cls = wk["cls"]
        keys = wk["k128"]
        worst, worst_big, n, n_small, wq = 0.0, 0.0, 0, 0, None
        n_drop, drop_max = 0, 0.0
        for name, ref in gold.items():
            parts = name.split("_")
            if parts[0] != "c%d" % cls:
                continue
            qd = [int(v) for v in parts[1:]]
            hit = np.flatnonzero(keys == ((qd[0] * 128 + qd[1]) * 128 + qd[2]) * 128 + qd[3])
            if len(hit) == 0:
                # dropped by the screen: it must be below the threshold
                n_drop += 1
                drop_max = max(drop_max, float(np.max(np.abs(ref))))
                continue
            i = int(hit[0])
            offs = wk["offs"]
            out = torch.empty(int(offs[i + 1] - offs[i]), dtype=torch.float64, device="cuda")
            f12int.eval_into(wk["Q"], wk["kern"], out, i, i + 1)
            got = out.cpu().numpy()
            mx = float(np.max(np.abs(ref)))
            scale = mx
            if cls == 5 and i5_vanishes(qd, shells):
                ref3 = gold["c3_%d_%d_%d_%d" % tuple(qd)]
                scale = float(np.max(shells[qd[0]].exps)) * float(np.max(np.abs(ref3)))
            err = float(np.max(np.abs(got - ref))) / scale
            n += 1
            if err > worst:
                worst, wq = err, {"quartet": qd, "max_abs_integral": mx}
            if mx >= 1e-12:
                worst_big = max(worst_big, err)
            else:
                n_small += 1
        res["I%d" % cls] = {"max_block_rel_err": worst, "worst_block": wq, "blocks": n,
                            "blocks_below_1e-12": n_small, "max_block_rel_err_blocks_above_1e-12": worst_big,
                            "sampled_blocks_dropped_by_screen": n_drop,
                            "largest_dropped_block": drop_max}
    f12int.stream_status()
    return res


# ---------------------------------------------------------------------------
def batched_main(args):
    """The batching workload: the 20-atom molecule (seed 5070) and two more of
    the same recipe and density (10 atoms in 9.5 bohr, seed 5071; 35 atoms in
    14.4 bohr, seed 5072), every unique quartet kept by the 1e-12 screen, all
    shapes from (ss|ss) to (ff|ff).  Lists are built on the device.  Step s
    takes slice (s + g) mod --slices of every shape group g of every list, and
    each class of a step runs as one launch of a captured graph (f12_batch:
    concurrent branches, tuned persistent contraction grids).  The plain path
    (per-shape launches on one stream, as the default workload runs) is timed
    on the same quartets."""
    import torch
    from paper_1412_5070_amd import f12int
    from synth import FACTOR_SETS, config_batching_extra, config_plain

    t_start = time.perf_counter()

    def log(msg):
        print("[bench %7.1fs] %s" % (time.perf_counter() - t_start, msg), file=sys.stderr, flush=True)

    P1 = FACTOR_SETS["P1"]
    (_, s10), (_, s35) = config_batching_extra()
    mols = [("20 atoms", config_plain()[1]), ("10 atoms", s10), ("35 atoms", s35)]
    classes = [int(c) for c in args.classes.split(",")]
    S = args.slices
    stream = torch.cuda.current_stream()
    tune_file = args.tune_file or os.path.join("/tmp", "f12_batch_tune_%d.txt" % os.getpid())
    geo = []
    for name, sh in mols:
        basis = f12int.Basis.from_shells(sh)
        geo.append((name, basis, f12int.Pairs(basis, 0)))
    steps_total = args.warmup + args.steps
    work = []
    for cls in classes:
        kern = f12int.Kernel(cls, P1, P1)
        kscr = f12int.Kernel(3, P1, P1) if cls == 5 else kern
        lists = []
        for (name, basis, pairs) in geo:
            Q = f12int.Quartets.build_device(pairs, pairs, cls, screen_tol=1e-12, screen_kernel=kscr)
            offs = Q.offsets()
            lists.append((Q, offs, name))
            log("I%d %s: %d quartets kept by the screen" % (cls, name, Q.n_quartets))
        work.append({"cls": cls, "kern": kern, "kscr": kscr, "lists": lists})

    ls_of = {}
    for wk in work:
        for (Q, offs, name) in wk["lists"]:
            ls_of[id(Q)] = Q.groups()[0]

    def step_parts(wk, step, ring):
        parts, pos = [], 0
        for (Q, offs, name) in wk["lists"]:
            starts = ls_of[id(Q)]
            for g in range(len(starts) - 1):
                a, b = int(starts[g]), int(starts[g + 1])
                n = b - a
                sl = (step + g) % S
                s0, s1 = a + (n * sl) // S, a + (n * (sl + 1)) // S
                if s1 <= s0:
                    continue
                size = int(offs[s1] - offs[s0])
                parts.append((Q, s0, s1, ring[pos:pos + size]))
                pos += size
        assert pos <= ring.numel()
        return parts

    # output buffer per class: the largest step of that class
    for wk in work:
        need = 0
        for step in range(steps_total):
            tot = 0
            for (Q, offs, name) in wk["lists"]:
                starts = ls_of[id(Q)]
                for g in range(len(starts) - 1):
                    a, b = int(starts[g]), int(starts[g + 1])
                    sl = (step + g) % S
                    s0, s1 = a + ((b - a) * sl) // S, a + ((b - a) * (sl + 1)) // S
                    tot += int(offs[s1] - offs[s0])
            need = max(need, tot)
        wk["ring"] = torch.empty(max(need, 1), dtype=torch.float64, device="cuda")
        wk["batches"] = []
        for step in range(steps_total):
            parts = step_parts(wk, step, wk["ring"])
            t0 = time.perf_counter()
            bt = f12int.Batch(parts, wk["kern"], nbranch=args.branches, tune=True, tune_path=tune_file)
            wk["batches"].append((bt, parts))
            log("I%d step %d: batch of %d quartets, %d parts, %d chunks (%.1f s to build)"
                % (wk["cls"], step, bt.n_quartets, len(parts), bt.n_chunks, time.perf_counter() - t0))

    def run(step, batched, rec):
        for wk in work:
            bt, parts = wk["batches"][step]
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if batched:
                bt.launch(stream)
            else:
                for (Q, s0, s1, out) in parts:
                    f12int.eval_into(Q, wk["kern"], out, s0, s1, stream)
            e1.record(stream)
            if rec is not None:
                rec.append((wk["cls"], bt.n_quartets, e0, e1))
        torch.cuda.synchronize()

    res = {}
    for mode in ("batched", "plain"):
        for w in range(args.warmup):
            run(w, mode == "batched", None)
        f12int.stream_status()
        rec = []
        t0 = time.perf_counter()
        for s_ in range(args.steps):
            run(args.warmup + s_, mode == "batched", rec)
            log("%s step %d done" % (mode, s_))
        elapsed = time.perf_counter() - t0
        f12int.stream_status()
        nq = sum(n for (_, n, _, _) in rec)
        per = {}
        for (cls, n, e0, e1) in rec:
            d = per.setdefault("I%d" % cls, [0, 0.0])
            d[0] += n
            d[1] += e0.elapsed_time(e1) / 1e3
        res[mode] = {"value": nq / elapsed, "elapsed": elapsed, "nq": nq,
                     "per_class": {k: v[0] / v[1] for k, v in per.items()}}
    grids = {}
    wk0 = work[0]
    for lab in range(7):
        for lcd in range(7):
            for i5 in (0, 1):
                for wk in work:
                    try:
                        grids["%d_%d_%s" % (lab, lcd, "I5" if i5 else "")] = wk["batches"][0][0].grid(lab, lcd, i5)
                        break
                    except f12int.F12Error:
                        pass
    line = {
        "metric": METRIC,
        "value": res["batched"]["value"],
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["batched"]["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batching: the 20-atom (seed 5070), 10-atom (seed 5071) and 35-atom (seed 5072) "
                        "molecules, s,s,p,p,d,f shells with 1-6 primitives, every unique quartet kept by "
                        "the 1e-12 screen, I2-I6 (factor P1); each step takes 1/%d of every shape group "
                        "of every list and runs each class as one captured graph (%d branches, tuned "
                        "persistent grids)" % (S, args.branches),
            "classes": ["I%d" % c for c in classes],
            "quartets_in_lists": {"I%d" % wk["cls"]: {name: Q.n_quartets for (Q, _, name) in wk["lists"]}
                                  for wk in work},
            "quartets_per_step": res["batched"]["nq"] // max(args.steps, 1),
        },
        "per_class_quartets_per_s": res["batched"]["per_class"],
        "plain_path_same_quartets": {"value": res["plain"]["value"], "per_class": res["plain"]["per_class"]},
        "speedup_vs_plain": res["batched"]["value"] / res["plain"]["value"],
        "tuned_contraction_grids": grids,
    }
    print(json.dumps(line))


def precision_main(args):
    """The precision workload: the 35-atom molecule (seed 5072, 14.4 bohr),
    every unique quartet kept by the 1e-12 screen, I2-I6 (P1), lists built on
    the device.  Step s takes slice (s + g) mod --slices of every shape group
    g; each step is evaluated with the FP64 contraction and with the
    split-FP32 ket transform (f12_eval_precision) on the same quartets.  The
    split result is compared with the FP64 one block by block over every
    evaluated block, and both with the stored oracle values of quartets
    sampled from the same molecule (tests/golden/prec35.npz)."""
    import torch
    from paper_1412_5070_amd import f12int
    from synth import FACTOR_SETS, config_precision

    t_start = time.perf_counter()

    def log(msg):
        print("[bench %7.1fs] %s" % (time.perf_counter() - t_start, msg), file=sys.stderr, flush=True)

    P1 = FACTOR_SETS["P1"]
    _, shells = config_precision()
    classes = [int(c) for c in args.classes.split(",")]
    S = args.slices
    stream = torch.cuda.current_stream()
    basis = f12int.Basis.from_shells(shells)
    pairs = f12int.Pairs(basis, 0)
    lsh = np.array([sh.l for sh in shells])
    _, cidx = np.unique(np.round(np.array([sh.center for sh in shells]), 12), axis=0, return_inverse=True)
    cidx = cidx.ravel()
    gold = {}
    gpath = os.path.join(ROOT, "tests", "golden", "prec35.npz")
    if os.path.exists(gpath):
        with np.load(gpath, allow_pickle=False) as z:
            gold = {k: z[k] for k in z.files}
    res, totals = {}, {}
    for cls in classes:
        kern = f12int.Kernel(cls, P1, P1)
        kscr = f12int.Kernel(3, P1, P1) if cls == 5 else kern
        Q = f12int.Quartets.build_device(pairs, pairs, cls, screen_tol=1e-12, screen_kernel=kscr)
        offs = Q.offsets()
        starts, _ = Q.groups()
        quads_all = Q.quads().astype(np.int64)
        log("I%d: %d quartets kept by the screen" % (cls, Q.n_quartets))
        steps = []
        for step in range(args.warmup + args.steps):
            parts = []
            for g in range(len(starts) - 1):
                a, b = int(starts[g]), int(starts[g + 1])
                sl = (step + g) % S
                s0, s1 = a + ((b - a) * sl) // S, a + ((b - a) * (sl + 1)) // S
                if s1 > s0:
                    parts.append((s0, s1))
            steps.append(parts)
        size = max(sum(int(offs[s1] - offs[s0]) for (s0, s1) in parts) for parts in steps)
        o64 = torch.empty(max(size, 1), dtype=torch.float64, device="cuda")
        o32 = torch.empty_like(o64)
        rc = {"fp64": [0, 0.0], "split_fp32": [0, 0.0]}
        worst_vs64 = 0.0
        nblocks = 0
        for step, parts in enumerate(steps):
            timed = step >= args.warmup
            for prec, out, key in ((0, o64, "fp64"), (1, o32, "split_fp32")):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                pos = 0
                for (s0, s1) in parts:
                    n = int(offs[s1] - offs[s0])
                    f12int.eval_precision(Q, kern, out[pos:pos + n], prec, s0, s1, stream)
                    pos += n
                e1.record(stream)
                torch.cuda.synchronize()
                if timed:
                    rc[key][0] += sum(s1 - s0 for (s0, s1) in parts)
                    rc[key][1] += e0.elapsed_time(e1) / 1e3
            if timed:
                # block-relative error of the split result against FP64, every block of the step
                # except those that vanish identically (their FP64 values are rounding noise):
                # one-centre blocks of odd l_a + l_b + l_c + l_d, and for I5 the blocks of
                # i5_vanishes (one shell twice as the bra, and the shell s or p or the ket two
                # s shells on its centre)
                qs = np.concatenate([quads_all[s0:s1] for (s0, s1) in parts])
                one_centre = (cidx[qs[:, 0]] == cidx[qs[:, 1]]) & (cidx[qs[:, 0]] == cidx[qs[:, 2]]) & \
                    (cidx[qs[:, 0]] == cidx[qs[:, 3]])
                vanish = one_centre & (lsh[qs].sum(axis=1) % 2 == 1)
                if cls == 5:
                    same = qs[:, 0] == qs[:, 1]
                    on_bra = (cidx[qs[:, 2]] == cidx[qs[:, 0]]) & (cidx[qs[:, 3]] == cidx[qs[:, 0]])
                    vanish |= same & ((lsh[qs[:, 0]] <= 1) | ((lsh[qs[:, 2]] == 0) & (lsh[qs[:, 3]] == 0) & on_bra))
                lens = np.concatenate([np.diff(offs[s0:s1 + 1]) for (s0, s1) in parts])
                lt = torch.as_tensor(lens, device="cuda")
                idx = torch.repeat_interleave(torch.arange(len(lens), device="cuda"), lt)
                n = int(lens.sum())
                scale = torch.zeros(len(lens), dtype=torch.float64, device="cuda").scatter_reduce_(
                    0, idx, o64[:n].abs(), "amax")
                diff = torch.zeros_like(scale).scatter_reduce_(0, idx, (o32[:n] - o64[:n]).abs(), "amax")
                ok = (scale > 0) & ~torch.as_tensor(vanish, device="cuda")
                worst_vs64 = max(worst_vs64, float((diff[ok] / scale[ok]).max()) if bool(ok.any()) else 0.0)
                nblocks += len(lens)
            log("I%d step %d done" % (cls, step))
        # stored oracle sample
        keys = None
        worst_or = {"fp64": 0.0, "split_fp32": 0.0}
        worst_blk = {"fp64": None, "split_fp32": None}
        nor, ndrop = 0, 0
        if gold:
            quads = quads_all
            keys = ((quads[:, 0] * 256 + quads[:, 1]) * 256 + quads[:, 2]) * 256 + quads[:, 3]
            for name, ref in gold.items():
                parts_ = name.split("_")
                if parts_[0] != "c%d" % cls:
                    continue
                qd = [int(v) for v in parts_[1:]]
                hit = np.flatnonzero(keys == ((qd[0] * 256 + qd[1]) * 256 + qd[2]) * 256 + qd[3])
                if len(hit) == 0:
                    ndrop += 1
                    continue
                i = int(hit[0])
                for prec, key in ((0, "fp64"), (1, "split_fp32")):
                    out = torch.empty(int(offs[i + 1] - offs[i]), dtype=torch.float64, device="cuda")
                    f12int.eval_precision(Q, kern, out, prec, i, i + 1, stream)
                    got = out.cpu().numpy()
                    sc = float(np.max(np.abs(ref)))
                    if cls == 5 and i5_vanishes(qd, shells):
                        continue
                    e = float(np.max(np.abs(got - ref))) / sc
                    if e > worst_or[key]:
                        worst_or[key] = e
                        worst_blk[key] = {"quartet": qd, "max_abs_integral": sc}
                nor += 1
            del quads, keys
        f12int.stream_status()
        res["I%d" % cls] = {
            "quartets_in_list": Q.n_quartets,
            "fp64_quartets_per_s": rc["fp64"][0] / rc["fp64"][1],
            "split_fp32_quartets_per_s": rc["split_fp32"][0] / rc["split_fp32"][1],
            "split_vs_fp64_max_block_rel_err": worst_vs64, "blocks_compared_with_fp64": nblocks,
            "vs_stored_oracle": {"blocks": nor, "sampled_blocks_dropped_by_screen": ndrop,
                                 "fp64_max_block_rel_err": worst_or["fp64"],
                                 "fp64_worst_block": worst_blk["fp64"],
                                 "split_fp32_max_block_rel_err": worst_or["split_fp32"],
                                 "split_fp32_worst_block": worst_blk["split_fp32"]}}
        totals[cls] = (rc["split_fp32"][0], rc["split_fp32"][1], rc["fp64"][0], rc["fp64"][1])
        del Q, quads_all
    line = {
        "metric": METRIC,
        "value": sum(v[0] for v in totals.values()) / sum(v[1] for v in totals.values()),
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 + split-f32 ket transform",
        "data": "synthetic",
        "config": {"workload": "precision: 35 atoms in a 14.4 bohr cube (seed 5072), s,s,p,p,d,f shells with 1-6 "
                               "primitives, every unique quartet kept by the 1e-12 screen, I2-I6 (factor P1); "
                               "each step 1/%d of every shape group, FP64 and split-FP32 contraction on the "
                               "same quartets" % S},
        "per_class": res,
        "fp64_value": sum(v[2] for v in totals.values()) / sum(v[3] for v in totals.values()),
        "note": "value: split-FP32 quartets/s over all timed steps of all classes; fp64_value: the FP64 "
                "contraction on the same quartets",
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batches", type=int, default=16)
    ap.add_argument("--classes", default=",".join(str(c) for c in CLASSES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--screen-tol", type=float, default=1e-12,
                    help="quartet screening threshold of the workload (0: every unique quartet)")
    ap.add_argument("--concurrent", action="store_true",
                    help="one stream per class, classes run concurrently (per-class rates then overlap)")
    ap.add_argument("--pipeline", action="store_true",
                    help="run the next slice's radial derivatives on a second stream while the current "
                         "slice contracts (launch timings then overlap)")
    ap.add_argument("--workload", choices=("plain", "batched", "precision"), default="plain",
                    help="plain: the 20-atom molecule through per-shape launches (default); batched: the "
                         "20-, 10- and 35-atom molecules, each class in one captured graph per step")
    ap.add_argument("--slices", type=int, default=64, help="batched: steps that cover the whole job")
    ap.add_argument("--branches", type=int, default=4, help="batched: concurrent branches of each graph")
    ap.add_argument("--tune-file", default=None, help="batched: tuning results to read and update")
    ap.add_argument("--chunk-log", default=None, metavar="FILE",
                    help="write one JSON line per timed output chunk (class, batch, quartet range, digest)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (three times) and exit: "
                         "the reference reading that scales the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the integral path has no multi-GPU mode; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload == "batched":
        batched_main(args)
        return
    if args.workload == "precision":
        precision_main(args)
        return

    import torch
    from paper_1412_5070_amd import f12int
    from synth import FACTOR_SETS, config_plain

    t_start = time.perf_counter()

    def log(msg):
        print("[bench %7.1fs] %s" % (time.perf_counter() - t_start, msg), file=sys.stderr, flush=True)

    classes = [int(c) for c in args.classes.split(",")]
    P1 = FACTOR_SETS["P1"]
    _, shells = config_plain()
    ls = np.array([s.l for s in shells])
    ks = np.array([len(s.exps) for s in shells])
    basis = f12int.Basis.from_shells(shells)
    pairs = f12int.Pairs(basis, 0)
    stream = torch.cuda.current_stream()

    # per class: quartet list, kernel, slices of every (la,lb,lc,ld) group
    work = []
    for cls in classes:
        kern = f12int.Kernel(cls, P1, P1)
        kscr = None
        if args.screen_tol > 0:
            kscr = f12int.Kernel(3, P1, P1) if cls == 5 else kern
        Q = f12int.Quartets.build(pairs, pairs, cls, screen_tol=args.screen_tol, screen_kernel=kscr)
        quads = Q.quads()
        offs = Q.offsets()
        key = ((ls[quads[:, 0]] * 4 + ls[quads[:, 1]]) * 4 + ls[quads[:, 2]]) * 4 + ls[quads[:, 3]]
        starts = np.concatenate([[0], np.nonzero(np.diff(key))[0] + 1, [len(key)]])
        nprim = ks[quads].prod(axis=1).astype(np.int64)
        nbra = (ks[quads[:, 0]] * ks[quads[:, 1]]).astype(np.int64)
        cprim = np.concatenate([[0], np.cumsum(nprim)])
        cbra = np.concatenate([[0], np.cumsum(nbra)])
        cap = f12int.scratch_prims(Q)
        groups = []
        for g in range(len(starts) - 1):
            a, b = int(starts[g]), int(starts[g + 1])
            la, lb, lc, ld = (int(ls[quads[a, i]]) for i in range(4))
            groups.append((a, b, (la, lb, lc, ld)))
        # a second copy of the list owns a second radial-derivative scratch, so
        # that slice s+1's derivatives can run while slice s contracts
        Q2 = (f12int.Quartets.build(pairs, pairs, cls, screen_tol=args.screen_tol, screen_kernel=kscr)
              if args.pipeline else None)
        work.append(dict(cls=cls, kern=kern, Q=Q, Q2=Q2, offs=offs, groups=groups, cprim=cprim, cbra=cbra,
                         spans=kernel_chains(kern.terms()),
                         cap=cap, nq=len(key), quads_all=quads,
                         k128=((quads[:, 0].astype(np.int64) * 128 + quads[:, 1]) * 128 + quads[:, 2]) * 128
                         + quads[:, 3]))
        log("I%d: %d quartets in %d groups" % (cls, len(key), len(groups)))

    # output rings in HBM, one per class (each class's stream writes its own)
    ring_all = torch.empty(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB
    per = ring_all.numel() // len(work)
    for i, wk in enumerate(work):
        wk["ring"] = ring_all[i * per:(i + 1) * per]
        wk["ring_pos"] = 0
        wk["stream"] = torch.cuda.Stream() if args.concurrent else stream
        wk["aux_stream"] = torch.cuda.Stream() if args.pipeline else wk["stream"]

    def slices(wk, batch):
        # groups are ordered by decreasing primitive count, so batch b takes
        # slice (b + g) mod batches of group g: every step mixes heavy and
        # light slices
        for g, (a, b, lq) in enumerate(wk["groups"]):
            n = b - a
            sl = (batch + g) % args.batches
            s0 = a + (n * sl) // args.batches
            s1 = a + (n * (sl + 1)) // args.batches
            while s0 < s1:
                # split so that a slice's primitive quartets fit the scratch
                hi = int(np.searchsorted(wk["cprim"], wk["cprim"][s0] + wk["cap"], side="right")) - 1
                e = max(s0 + 1, min(s1, hi))
                yield s0, e, lq
                s0 = e

    def run_step(batch, record):
        start = torch.cuda.Event()
        start.record(stream)
        for wk in work:
            Q, kern, offs = wk["Q"], wk["kern"], wk["offs"]
            st = wk["stream"]
            st.wait_event(start)
            ev_cls0 = torch.cuda.Event(enable_timing=True)
            ev_cls1 = torch.cuda.Event(enable_timing=True)
            ev_cls0.record(st)
            nq = 0
            ring = wk["ring"]
            sa = wk["aux_stream"]
            sa.wait_event(ev_cls0)
            done = [None, None]  # last contraction that read each list's scratch
            for i, (s0, s1, lq) in enumerate(slices(wk, batch)):
                size = int(offs[s1] - offs[s0])
                if wk["ring_pos"] + size > ring.numel():
                    wk["ring_pos"] = 0
                out = ring[wk["ring_pos"]:wk["ring_pos"] + size]
                wk["ring_pos"] += size
                Qi = Q if (wk["Q2"] is None or i % 2 == 0) else wk["Q2"]
                if done[i % 2] is not None and sa is not st:
                    sa.wait_event(done[i % 2])
                ea = torch.cuda.Event(enable_timing=True)
                ea_end = torch.cuda.Event(enable_timing=True)
                ea.record(sa)
                f12int.eval_stage(Qi, kern, out, s0, s1, 1, sa)
                ea_end.record(sa)
                if sa is not st:
                    st.wait_event(ea_end)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                f12int.eval_stage(Qi, kern, out, s0, s1, 2, st)
                e1.record(st)
                done[i % 2] = e1
                # the chunk's checksum (read back after the timed steps)
                if record is not None:
                    slot = len(record["chunks"])
                    dslot = digests[slot:slot + 1]
                else:
                    dslot = digest_sink
                ed1 = torch.cuda.Event(enable_timing=True)
                f12int.digest(Qi, out, dslot, s0, s1, st)
                ed1.record(st)
                if record is not None:
                    record["chunks"].append((wk["cls"], batch, s0, s1, e1, ed1, 8 * size))
                if record is not None:
                    record["aux"].append((ea, ea_end))
                nq += s1 - s0
                if record is not None:
                    la, lb, lc, ld = lq
                    i5 = wk["cls"] == 5
                    npq = int(wk["cprim"][s1] - wk["cprim"][s0])
                    nbp = int(wk["cbra"][s1] - wk["cbra"][s0])
                    fl = method_flops(la, lb, lc, ld, i5, npq, nbp)
                    flf = contraction_flops(la, lb, lc, ld, i5, npq, nbp, s1 - s0)
                    L = la + lb + lc + ld + (2 if i5 else 0)
                    # algorithmic HBM bytes: blocks written, A_0..A_L read, four list entries per quartet
                    nbytes = 8 * size + 8 * (L + 1) * npq + 32 * (s1 - s0)
                    record["launches"].append((kernel_name(la, lb, lc, ld, i5), fl, e0, e1, nbytes, flf))
                    record["aux_flops"].append(aux_flops(L, wk["spans"], npq))
            ev_cls1.record(st)
            if record is not None:
                record["classes"].append((wk["cls"], nq, ev_cls0, ev_cls1))
            if not args.concurrent:
                torch.cuda.synchronize()
                log("batch %d I%d: %d quartets done" % (batch, wk["cls"], nq))
        torch.cuda.synchronize()
        log("batch %d: all classes done" % batch)

    # one 64-bit digest per timed output chunk (f12_digest adds into its slot)
    n_chunks = sum(1 for s in range(args.steps) for wk in work
                   for _ in slices(wk, (args.warmup + s) % args.batches))
    digests = torch.zeros(max(n_chunks, 1), dtype=torch.int64, device="cuda")
    digest_sink = torch.zeros(1, dtype=torch.int64, device="cuda")

    for w in range(args.warmup):
        run_step(w % args.batches, None)
    torch.cuda.synchronize()
    f12int.stream_status()
    rec = {"launches": [], "classes": [], "aux": [], "aux_flops": [], "chunks": []}
    t0 = time.perf_counter()
    nq_total = 0
    for s in range(args.steps):
        batch = (args.warmup + s) % args.batches
        run_step(batch, rec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    f12int.stream_status()
    nq_total = sum(n for (_, n, _, _) in rec["classes"])

    per_class = {}
    for (cls, n, e0, e1) in rec["classes"]:
        d = per_class.setdefault("I%d" % cls, [0, 0.0])
        d[0] += n
        d[1] += e0.elapsed_time(e1) / 1e3
    per_class_rate = {k: v[0] / v[1] for k, v in per_class.items()}

    by_kernel = {}
    alg_bytes = 0
    fl_fact = 0.0
    for (name, fl, e0, e1, nb, flf) in rec["launches"]:
        d = by_kernel.setdefault(name, [0, 0.0, 0.0])
        d[0] += 1
        d[1] += fl
        d[2] += e0.elapsed_time(e1) / 1e3
        alg_bytes += nb
        fl_fact += flf
    dom = max(by_kernel, key=lambda k: by_kernel[k][2])
    n_c = sum(v[0] for v in by_kernel.values())
    fl_c = sum(v[1] for v in by_kernel.values())
    contraction_time = sum(v[2] for v in by_kernel.values())
    achieved = fl_c / contraction_time / 1e12
    aux_time = sum(a.elapsed_time(b) / 1e3 for (a, b) in rec["aux"])
    aux_fl = float(sum(rec["aux_flops"]))
    gpu_time = sum(v[1] for v in per_class.values())

    # chunk digests: per class the sum mod 2^64 (equal to the digest of all the
    # class's timed blocks); the digest launch is timed from the end of the
    # contraction that wrote the chunk to its own end
    dg = digests[:len(rec["chunks"])].cpu().numpy().view(np.uint64)
    per_class_digest = {}
    for (cls, _, _, _, _, _, _), v in zip(rec["chunks"], dg):
        per_class_digest[cls] = (per_class_digest.get(cls, 0) + int(v)) % 2 ** 64
    dig_time = sum(a.elapsed_time(b) / 1e3 for (_, _, _, _, a, b, _) in rec["chunks"])
    dig_bytes = sum(nb for (_, _, _, _, _, _, nb) in rec["chunks"])
    big = [(a.elapsed_time(b) / 1e3, nb) for (_, _, _, _, a, b, nb) in rec["chunks"] if nb >= 32 << 20]
    if args.chunk_log:
        with open(args.chunk_log, "w") as fh:
            for (cls, batch, s0, s1, _, _, nb), v in zip(rec["chunks"], dg):
                fh.write(json.dumps({"class": "I%d" % cls, "batch": batch, "q_begin": s0, "q_end": s1,
                                     "doubles": nb // 8, "digest": "%016x" % int(v)}) + "\n")

    log("stored oracle sample")
    accuracy = stored_sample_errors(work, shells)

    rec_ok = TRAFFIC_RECORD["sources_sha1"] == kernel_sources_sha1()
    traffic = TRAFFIC_RECORD["contraction_bytes_per_launch"] if rec_ok else None
    aux_traffic = TRAFFIC_RECORD["aux_bytes_per_launch"] if rec_ok else None

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle sample")
        cb = cpu_baseline(work, ks)
        log("CPU oracle: %.3g quartets/s on %d cores" % (cb["rate"], cb["cores"]))
        cpu = {"value": cb["rate"], "unit": "quartets/s", "cores": cb["cores"], "kind": "oracle",
               "value_one_core": cb["rate_one_core"],
               "sample": "stratified by class (I2-I6) and primitive-count bin (1-4, 5-16, 17-64): %d quartets "
                         "drawn uniformly per stratum from the 20-atom lists, %.0f s of CPU work in one worker "
                         "process per core; stratum mean times weighted by the workload's quartet counts. "
                         "Quartets with more than 64 primitive quartets are not sampled: the strata hold "
                         "%.1f%% of the workload's quartets" % (cb["quartets_timed"], cb["cpu_seconds"],
                                                                100 * cb["coverage"]),
               "strata": cb["strata"]}

    line = {
        "metric": METRIC,
        "value": nq_total / elapsed,
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "20 atoms in a 12 bohr cube (seed 5070), s,s,p,p,d,f shells with 1-6 "
                        "primitives, %s of I2-I6 (factor P1), one of %d stratified batches per step"
                        % ("the unique quartets kept by the %.0e screen" % args.screen_tol if args.screen_tol > 0
                           else "all unique quartets", args.batches),
            "screen_tol": args.screen_tol,
            "quartets_in_lists": {"I%d" % wk["cls"]: wk["nq"] for wk in work},
            "classes": ["I%d" % c for c in classes],
            "streams": ("one per class, concurrent (per-class rates overlap)" if args.concurrent else "one")
                       + ("; radial derivatives of the next slice overlap the contraction" if args.pipeline else ""),
            "quartets_per_step": nq_total // max(args.steps, 1),
        },
        "per_class_quartets_per_s": per_class_rate,
        "roofline": {
            "kernel": "E.R.E contraction (big_kernel<*>)",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE x %.4f + WRITE_SIZE x %.4f)"
                            % (TRAFFIC_RECORD["fetch_scale"], TRAFFIC_RECORD["write_scale"]),
            "flops_per_launch_count": "method count: per primitive quartet 3 C(L+4,4) (R) + 2 H_ab H_cd n_cd "
                                      "(ket); per bra primitive pair 2 n_ab H_ab n_cd x E^ab nonzero fraction "
                                      "(bra); I5 4x ket and bra, R at L+2",
            "factorised_passes": {"flops_per_launch": fl_fact / n_c,
                                  "achieved": fl_fact / contraction_time / 1e12,
                                  "frac": fl_fact / contraction_time / 1e12 / FP64_VECTOR_PEAK_TFLOPS},
            "algorithmic_bytes_per_launch": alg_bytes / n_c,
            "hardware_fp64": None if not rec_ok else {
                "flops_per_launch": TRAFFIC_RECORD["contraction_hw_fp64_flops_per_launch"],
                "achieved": TRAFFIC_RECORD["contraction_hw_fp64_flops_per_launch"] / (contraction_time / n_c) / 1e12,
                "frac": TRAFFIC_RECORD["contraction_hw_fp64_flops_per_launch"] / (contraction_time / n_c) / 1e12
                        / FP64_VECTOR_PEAK_TFLOPS},
            "launches": n_c,
            "avg_launch_ms": contraction_time / n_c * 1e3,
            "flops_per_launch": fl_c / n_c,
            "share_of_gpu_time": contraction_time / gpu_time,
            "largest_instantiation": {
                "kernel": dom, "launches": by_kernel[dom][0],
                "avg_launch_ms": by_kernel[dom][2] / by_kernel[dom][0] * 1e3,
                "achieved": by_kernel[dom][1] / by_kernel[dom][2] / 1e12},
            "aux_kernel": {"launches": len(rec["aux"]), "avg_launch_ms": aux_time / max(len(rec["aux"]), 1) * 1e3,
                           "share_of_gpu_time": aux_time / gpu_time, "traffic": aux_traffic,
                           "flops_per_launch": aux_fl / max(len(rec["aux"]), 1),
                           "achieved": aux_fl / aux_time / 1e12,
                           "frac": aux_fl / aux_time / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                           "flops_count": "per chain and sign a ladder start (%d flops) + 6 (L + span); per sign "
                                          "8 (L+1)(L+2)(2L+3)/6 for the radial-derivative recursion"
                                          % AUX_START_FLOPS,
                           "hardware_fp64_achieved": None if not rec_ok else
                           TRAFFIC_RECORD["aux_hw_fp64_flops_per_launch"] / (aux_time / max(len(rec["aux"]), 1)) / 1e12},
        },
        "output_digest": {
            "kernel": "chunk checksum (f12_digest), one launch per output chunk",
            "per_class": {"I%d" % c: "%016x" % v for c, v in sorted(per_class_digest.items())},
            "chunks": len(rec["chunks"]),
            "avg_launch_ms": dig_time / max(len(rec["chunks"]), 1) * 1e3,
            "bytes_per_launch": dig_bytes / max(len(rec["chunks"]), 1),
            "achieved_GBps": dig_bytes / max(dig_time, 1e-30) / 1e9,
            "frac_of_hbm_peak": dig_bytes / max(dig_time, 1e-30) / 1e9 / HBM_PEAK_GBPS,
            "share_of_gpu_time": dig_time / gpu_time,
            "chunks_of_32MiB_or_more": {
                "chunks": len(big),
                "achieved_GBps": sum(nb for _, nb in big) / max(sum(t for t, _ in big), 1e-30) / 1e9,
                "frac_of_hbm_peak": sum(nb for _, nb in big) / max(sum(t for t, _ in big), 1e-30) / 1e9
                                    / HBM_PEAK_GBPS},
        },
        "accuracy_vs_stored_oracle": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
