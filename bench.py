"""Benchmark: K elements/s of the MASTER coupling matrices K^TT, K^TE, K^EE,
K^BB at lmax = 6000 on one MI355X, with the roofline of the l3-reduction
kernel and the CPU oracle timed on a bounded sample beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32c|both]

A step is one couple_matrix call (window scaling -> l3 reduction -> fill) for
all four spectra of the synthetic lmax = 6000 window (inputs resident in HBM,
output 4 x 6001^2 float64 written to HBM).  The timed region is bracketed by
torch.cuda.synchronize() on both sides; per-kernel durations come from HIP
events the library records on the call's stream.  One JSON line is printed.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ALU peaks, 256 CU x 2.4 GHz x 2 FLOP per FMA lane: fp64 64 lanes/clk/CU (78.6 TFLOP/s);
# fp32 128 lanes/clk/CU (157.3 TFLOP/s), reached on gfx950 by plain (non-packed) fp32 VALU ops.
PEAK_VALU_TFLOPS = {"fp64": 78.6, "fp32c": 157.3}
PEAK_HBM_GBS = 8000.0
# Useful arithmetic per even-L triple as the strip kernels evaluate it (FMA = 2 FLOP): the
# (0 0 0)^2 factors g(k) g(d+k) W'(l3) are wave-uniform per step and folded into U(k), so
# per triple TT is P = g h (1) and one FMA (2); TE/EE are N' (one add and one FMA: 3),
# y = P N' and z = y N' (2) and two FMA accumulations (4).  This is the roofline's
# achieved rate.
FLOP_PER_TRIPLE_POL = 12
# The method's count with X^2 formed per triple (three multiplies), as the paper's
# evaluation of eq. 000_sq_main does: TT 5 + TE/EE 11.  Reported as the effective rate.
FLOP_PER_TRIPLE_PAPER = 16
# The band-limited call asks for TT, EE and BB only, so the strip runs without the TE
# accumulation: 12 - 2.
FLOP_PER_TRIPLE_BAND = 10


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "strip_pol4_lmax6000_traffic.md")
STRIP_SOURCES = [os.path.join(ROOT, "paper_2602_15605_amd", "csrc", f) for f in ("strip.hip", "strip_params.hpp")]


def measured_traffic(kernel: str):
    """HBM bytes per launch of a strip kernel from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None when it is missing or the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for path in STRIP_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    value = digest = None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch %s =" % kernel):
            value = int(line.split("=")[1])
        if line.startswith("kernel_source_sha256"):
            digest = line.split("=")[1].strip()
    return value if digest == h.hexdigest() else None


def band_triples(lmax: int, cut: int) -> int:
    """Even-L triples with l1 <= l2 <= lmax and l3 <= cut (the band-limited sum)."""
    total = 0
    for d in range(0, min(cut, lmax) + 1):
        l1 = np.arange(0, lmax - d + 1, dtype=np.int64)
        top = np.minimum(2 * l1 + d, cut)
        total += int(np.sum((top - d) // 2 + 1))
    return total


def triples(lmax: int) -> int:
    """Even-L triples with l1 <= l2: C(lmax + 3, 3)."""
    return math.comb(lmax + 3, 3)


def bench_rows(lmax: int, n: int) -> np.ndarray:
    """Rows of the cpu_baseline sample and its error check: n - 4 seeded rows
    plus rows 0, 1, 2 and lmax (the longest rows are always in)."""
    from paper_2602_15605_amd import synth
    return synth.sample_rows(lmax, fraction=0.0, seed=6000, minimum=max(1, n - 4))


def te_plain_error(K, K_ref, A_ref, floor=1e-3):
    """Plain relative error |dK|/|K_ref| over the TE elements with |K_ref| >= floor A_ref."""
    big = (A_ref > 0) & (np.abs(K_ref) >= floor * A_ref)
    if not np.any(big):
        return 0.0
    return float(np.max(np.abs(K[big] - K_ref[big]) / np.abs(K_ref[big])))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_context(torch, couple, synth):
    """Context numbers beside the headline (never `value`):
    * the paper's own GPU comparison point: K^TT alone and K^EE alone at
      lmax = 10^4 in FP64 (the paper times each on an A100);
    * end to end at lmax = 6000, FP32C: couple_init (tables), W host -> device,
      couple_matrix, K device -> host (pageable), wall clock."""
    out = {}
    L = 10000
    W = [synth.window_spectrum(L, 2500.0, 9000 + s) for s in range(3)]   # a full (not band-limited) window
    ctx = couple.couple_init(L)
    dW = [torch.as_tensor(w).cuda() for w in W]
    res = torch.empty((1, L + 1, L + 1), dtype=torch.float64, device="cuda")
    for spec in ("TT", "EE"):
        args = [dW[0] if spec == "TT" else None, None, dW[2] if spec == "EE" else None]
        ms = _timed(torch, lambda: couple.couple_matrix(ctx, *args, L, spectra=(spec,), precision="fp64", out=res),
                    3, 1)
        out["single_spectrum_lmax10000_fp64_" + spec] = {
            "ms_per_call": ms, "k_elements_per_s": (L + 1) ** 2 / (ms * 1e-3),
            "note": "the paper times K^TT (0.63 s) and K^EE (3.2 s) at lmax=10^4 on an A100 (kernel only)"}
    del res
    couple.couple_free(ctx)
    torch.cuda.synchronize()
    lmax = 6000
    Wh = synth.workload_windows(2, lmax=lmax)
    t0 = time.perf_counter()
    ctx = couple.couple_init(lmax)
    dW = [torch.as_tensor(w).cuda() for w in Wh]
    K = couple.couple_matrix(ctx, *dW, lmax, spectra=("TT", "TE", "EE", "BB"), precision="fp32c")
    Kh = K.cpu()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["end_to_end_lmax6000_fp32c"] = {
        "ms": 1e3 * dt, "k_elements_per_s": 4 * (lmax + 1) ** 2 / dt,
        "includes": "couple_init (tables), W host->device, couple_matrix, 1.15 GB K device->host (pageable)"}
    del K, Kh
    # binned MASTER solve on these windows: bins of 50 from l = 2, TT and the E/B block
    edges = list(range(2, lmax + 2, 50)) + [lmax + 1]
    nb = len(edges) - 1
    Kt = couple.couple_band(ctx, 0, 2 * lmax, dW[0], None, None, lmax, spectra=("TT",), precision="fp32c",
                            bin_edges=edges)[0].contiguous()
    Kp = couple.couple_band(ctx, 0, 2 * lmax, None, None, dW[2], lmax, spectra=("EE", "BB", "EB"),
                            precision="fp32c", bin_edges=edges)
    cl = torch.ones((3, lmax + 1), dtype=torch.float64, device="cuda")
    wt = torch.empty(nb * (nb + 1), dtype=torch.float64, device="cuda")
    wp = torch.empty(2 * nb * (2 * nb + 1), dtype=torch.float64, device="cuda")
    ctb = torch.empty((3, nb), dtype=torch.float64, device="cuda")
    xt = torch.empty((1, nb), dtype=torch.float64, device="cuda")
    xp = torch.empty((1, 2 * nb), dtype=torch.float64, device="cuda")
    ms_t = _timed(torch, lambda: (couple.couple_bin_spectra(ctx, cl, edges, out=ctb),
                                  couple.couple_master_solve(ctx, Kt, ctb[0:1], work=wt, out=xt)), 5, 2)
    ms_p = _timed(torch, lambda: (couple.couple_bin_spectra(ctx, cl, edges, out=ctb),
                                  couple.couple_master_solve(ctx, Kp, ctb[1:3].reshape(1, -1), pol=True, work=wp,
                                                              out=xp)),
                  5, 2)
    # 3j rows from the tables: 2000 seeded pairs with l1, l2 <= 6000, every l3, each family
    rng = np.random.default_rng(6001)
    l1 = rng.integers(0, lmax + 1, 2000).astype(np.int32)
    l2 = rng.integers(0, lmax + 1, 2000).astype(np.int32)
    t1, t2 = torch.as_tensor(l1).cuda(), torch.as_tensor(l2).cuda()
    n_sym = int(np.sum(2 * np.minimum(l1, l2) + 1))
    rows = torch.empty((2000, 2 * lmax + 1), dtype=torch.float64, device="cuda")
    for m in (0, 1, 2):
        ms = _timed(torch, lambda: couple.couple_threej_rows(ctx, t1, t2, m, stride=2 * lmax + 1, out=rows), 5, 2)
        out["threej_rows_2000pairs_lmax6000_m%d" % m] = {
            "ms_per_call": ms, "symbols": n_sym, "symbols_per_s": n_sym / (ms * 1e-3),
            "note": "(l1 l2 l3; -m m 0) for every l3 of each pair, float64, rows padded to 12001"}
    for (m1, m2) in ((1, 1), (2, 2)):
        ms = _timed(torch, lambda: couple.couple_threej_rows_m(ctx, t1, t2, m1, m2, stride=2 * lmax + 1, out=rows),
                    5, 2)
        out["threej_rows_2000pairs_lmax6000_%d%d%d" % (m1, m2, -m1 - m2)] = {
            "ms_per_call": ms, "symbols": n_sym, "symbols_per_s": n_sym / (ms * 1e-3),
            "note": "(l1 l2 l3; %d %d %d) for every l3 of each pair, float64, exact 128-bit numerators" % (
                m1, m2, -m1 - m2)}
    del rows
    out["master_solve_lmax6000_bins50"] = {
        "bins": nb, "tt_ms": ms_t, "eb_block_ms": ms_p,
        "note": "binned pseudo-spectra + LU solve on one work-group; TT is %d unknowns, E/B %d" % (nb, 2 * nb)}
    # fine bins (width 3): TT 2000 unknowns, E/B 4000, on the multi-work-group path
    edges3 = list(range(2, lmax + 2, 3))
    if edges3[-1] != lmax + 1:
        edges3.append(lmax + 1)
    nb3 = len(edges3) - 1
    Kt3 = couple.couple_band(ctx, 0, 2 * lmax, dW[0], None, None, lmax, spectra=("TT",), precision="fp32c",
                             bin_edges=edges3)[0].contiguous()
    Kp3 = couple.couple_band(ctx, 0, 2 * lmax, None, None, dW[2], lmax, spectra=("EE", "BB", "EB"),
                             precision="fp32c", bin_edges=edges3)
    # right-hand sides of C_b = 1 in every bin: the row sums of the binned systems
    rt3 = Kt3.sum(dim=1).reshape(1, -1).contiguous()
    rp3 = torch.cat([Kp3[0].sum(dim=1) + Kp3[2].sum(dim=1), Kp3[2].sum(dim=1) + Kp3[1].sum(dim=1)]).reshape(1, -1)
    wt3 = torch.empty(nb3 * (nb3 + 1), dtype=torch.float64, device="cuda")
    wp3 = torch.empty(2 * nb3 * (2 * nb3 + 1), dtype=torch.float64, device="cuda")
    xt3 = torch.empty((1, nb3), dtype=torch.float64, device="cuda")
    xp3 = torch.empty((1, 2 * nb3), dtype=torch.float64, device="cuda")
    ms_t3 = _timed(torch, lambda: couple.couple_master_solve(ctx, Kt3, rt3, work=wt3, out=xt3), 3, 1)
    ms_p3 = _timed(torch, lambda: couple.couple_master_solve(ctx, Kp3, rp3.contiguous(), pol=True, work=wp3,
                                                             out=xp3), 3, 1)
    out["master_solve_lmax6000_bins3"] = {
        "bins": nb3, "tt_ms": ms_t3, "eb_block_ms": ms_p3,
        "max_abs_dev_from_1": {"tt": float((xt3 - 1.0).abs().max()), "eb": float((xp3 - 1.0).abs().max())},
        "note": "the solve alone, right-hand sides K 1, so C_b = 1 comes back; TT is %d unknowns, E/B %d, "
                "outer panels spread over the chip" % (nb3, 2 * nb3)}
    del Kt3, Kp3, wp3
    couple.couple_free(ctx)
    return out


def run_scaling(torch, couple, synth):
    """Strip time against lmax (Sec. 4.2 and Fig. 2 claim cubic scaling of the
    coupling computation): couple_matrix for all four spectra at lmax in
    linspace(500, 6000, 12) with the workload's windows, FP64 and FP32C.  Each
    point reports the call and strip times and triples/s; the fitted log-log
    slope of strip time against lmax is given over all points and over
    lmax >= 2000 (below, per-call overheads weigh in)."""
    out = {}
    lmaxes = [int(x) for x in np.linspace(500, 6000, 12)]
    ctx = couple.couple_init(max(lmaxes))
    spectra = ("TT", "TE", "EE", "BB")
    for prec in ("fp32c", "fp64"):
        pts = []
        for L in lmaxes:
            dW = [torch.as_tensor(w).cuda() for w in synth.workload_windows(2, lmax=L)]
            res = torch.empty((4, L + 1, L + 1), dtype=torch.float64, device="cuda")
            call = lambda: couple.couple_matrix(ctx, *dW, L, spectra=spectra, precision=prec, out=res)
            ms = _timed(torch, call, 5, 2)
            couple.couple_profile(ctx, True)
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            prof = couple.couple_profile_read(ctx)
            couple.couple_profile(ctx, False)
            strip = prof["strip"][0] / max(1, prof["strip"][1])
            pts.append({"lmax": L, "ms_per_call": ms, "strip_ms": strip,
                        "triples_per_s": triples(L) / (strip * 1e-3)})
            del res, dW
        x = np.log([p["lmax"] for p in pts])
        y = np.log([p["strip_ms"] for p in pts])
        big = np.array([p["lmax"] >= 2000 for p in pts])
        out[prec] = {"points": pts, "slope_all": float(np.polyfit(x, y, 1)[0]),
                     "slope_lmax_ge_2000": float(np.polyfit(x[big], y[big], 1)[0])}
        print("[bench] scaling %s: slope %.3f (all), %.3f (lmax >= 2000)" %
              (prec, out[prec]["slope_all"], out[prec]["slope_lmax_ge_2000"]), file=sys.stderr, flush=True)
    couple.couple_free(ctx)
    out["note"] = "the paper reports cubic scaling of the coupling computation with lmax (Sec. 4.2, Fig. 2)"
    return out


def run_extras(torch, couple, synth, args):
    """The band-limited and batched workloads, timed the same way (device time
    per call, inputs resident); reported beside the headline, not as it."""
    out = {}
    steps, warm = 8, 3
    # band-limited: lmax=10000, l3<=1000, 8 masks, TT/EE/BB, 200 bins of 50, FP32C
    L, cut = 10000, 1000
    ctx = couple.couple_init(L)
    masks = [synth.workload_windows(4, mask=m) for m in range(8)]
    dW = [[torch.as_tensor(masks[m][s]).cuda() for m in range(8)] for s in range(3)]
    edges = list(range(0, 10001, 50))
    res = torch.empty((8, 3, 200, 200), dtype=torch.float64, device="cuda")
    T_band = band_triples(L, cut)
    for prec in ("fp32c", "fp64"):
        call = lambda: couple.couple_band_batched(ctx, 0, cut, dW[0], None, dW[2], L, spectra=("TT", "EE", "BB"),
                                                  precision=prec, bin_edges=edges, out=res)
        ms = _timed(torch, call, steps, warm)
        couple.couple_profile(ctx, True)
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        prof = couple.couple_profile_read(ctx)
        couple.couple_profile(ctx, False)
        kms = {k: prof[k][0] / steps for k in ("scale_windows", "strip", "fill")}
        # TT and EE per triple (no TE): P, the TT FMA, the t step, the N' FMA, two multiplies, the EE FMA
        tflops = FLOP_PER_TRIPLE_BAND * T_band * 8 / (kms["strip"] * 1e-3) / 1e12
        # the multi-mask strip forms P, N' (3 FLOP; 4 in the wide float64 form) and the two
        # products once per term for its 4 masks, then 2 FMAs per mask: executed FLOP per
        # mask-triple = 4 + shared / 4
        shared = 1 + (3 if prec == "fp32c" else 4) + 2
        executed = 4 + shared / 4.0
        xtflops = executed * T_band * 8 / (kms["strip"] * 1e-3) / 1e12
        peak = PEAK_VALU_TFLOPS[prec]
        out["band_lmax10000_cut1000_8masks_binned_" + prec] = {
            "ms_per_call": ms, "masks": 8, "spectra": ["TT", "EE", "BB"], "bins": 200,
            "kernel_ms_per_call": kms, "launches_per_call": {k: prof[k][1] / steps for k in kms},
            "triples_per_mask": T_band, "flop_per_triple_executed": executed,
            "strip_tflops": xtflops, "strip_roofline_frac": xtflops / peak,
            "flop_per_triple_single_mask": FLOP_PER_TRIPLE_BAND,
            "strip_single_mask_equiv_tflops": tflops, "strip_single_mask_equiv_frac": tflops / peak,
            "note": ("two multi-mask strip launches of four masks (windows once per group), then one zero and "
                     "one bin launch per group; strip_tflops / strip_roofline_frac count the FLOP executed "
                     "(P, N' and the two products once per term for the group, 2 FMAs per mask); "
                     "strip_single_mask_equiv_* charge every mask the single-mask 10 FLOP per triple, "
                     "the rate one launch per mask would need to match")}
    # the same band-limited call writing the symmetric kernels Xi (the covariance kernels when
    # the windows are squared-mask spectra)
    ms = _timed(torch, lambda: couple.couple_band_batched(ctx, 0, cut, dW[0], None, dW[2], L,
                                                          spectra=("TT", "EE", "BB"), precision="fp32c",
                                                          bin_edges=edges, out=res, xi=True), steps, warm)
    out["band_lmax10000_cut1000_8masks_binned_xi_fp32c"] = {
        "ms_per_call": ms, "masks": 8, "spectra": ["TT", "EE", "BB"], "bins": 200, "output": "Xi"}
    # with the odd-L EB matrix: the multi-mask odd-L strip runs beside the even one; timed
    # against eight one-mask calls (the results are bitwise equal)
    pol = ("EE", "BB", "EB")
    res_pol = torch.empty((8, 3, 200, 200), dtype=torch.float64, device="cuda")
    for prec in ("fp32c", "fp64"):
        ms = _timed(torch, lambda: couple.couple_band_batched(ctx, 0, cut, None, None, dW[2], L, spectra=pol,
                                                              precision=prec, bin_edges=edges, out=res_pol),
                    steps, warm)

        def one_mask_calls():
            for m in range(8):
                couple.couple_band(ctx, 0, cut, None, None, dW[2][m], L, spectra=pol, precision=prec,
                                   bin_edges=edges, out=res_pol[m])

        ms_one = _timed(torch, one_mask_calls, steps, warm)
        out["band_lmax10000_cut1000_8masks_binned_eebbeb_" + prec] = {
            "ms_per_call": ms, "one_mask_calls_ms": ms_one, "masks": 8, "spectra": list(pol), "bins": 200}
    del res_pol
    couple.couple_free(ctx)
    del dW, res
    # batched: 32 masks, lmax uniform in [500, 4000], 4 spectra, matrix-core contraction
    lmaxes = [int(x) for x in synth.batched_lmaxes()]
    ctx = couple.couple_init(max(lmaxes))
    Ws = [synth.workload_windows(3, mask=m) for m in range(len(lmaxes))]
    dW = [[torch.as_tensor(w[s]).cuda() for w in Ws] for s in range(3)]
    outs = [torch.empty((4, L + 1, L + 1), dtype=torch.float64, device="cuda") for L in lmaxes]
    couple.couple_reserve_batched(ctx, lmaxes)
    n_el = sum(4 * (L + 1) ** 2 for L in lmaxes)
    # useful contraction FLOP: 2 per (pair, l3, mask, spectrum) over TT/TE/EE, each mask at its own lmax
    contraction = sum(2 * 3 * triples(L) for L in lmaxes)
    check_rows = None
    if not args.no_check:
        from oracle import bulk
        check_rows = [np.array(sorted({2, L // 2, L})) for L in lmaxes]
        refs = [bulk.coupling_rows(L, *Ws[m], rows=check_rows[m], spectra=("TT", "TE", "EE", "BB"))
                for m, L in enumerate(lmaxes)]
    for prec in ("mfma_fp32", "mfma_bf16x3", "fp32c"):
        call = lambda: couple.couple_matrix_batched(ctx, lmaxes, dW[0], dW[1], dW[2], precision=prec, outs=outs)
        r = {"masks": len(lmaxes), "elements": n_el}
        if prec == "mfma_bf16x3":
            r["accuracy_class"] = "2e-5 (bfloat16 hi/lo split, bound 3*2^-16 per term); not a 1e-6 mode"
        else:
            r["accuracy_class"] = "1e-6"
        if prec == "mfma_fp32":
            # useful contraction FLOP (each mask at its own lmax); the kernel runs 4-mask
            # tiles up to each tile's largest lmax, so at most three columns idle per tile
            r["useful_contraction_flop"] = contraction
        if prec.startswith("mfma"):
            tm, fl, tms = couple.couple_autotune_batched(ctx, lmaxes, dW[0], dW[1], dW[2], outs=outs,
                                                         precision=prec)
            r["tiles"] = {"row_tiles": tm, "flush": fl, "autotune_ms": tms}
        ms = _timed(torch, call, steps, warm)
        r.update({"ms_per_call": ms, "k_elements_per_s": n_el / (ms * 1e-3)})
        if prec.startswith("mfma"):
            couple.couple_profile(ctx, True)
            call()
            prof = couple.couple_profile_read(ctx)
            couple.couple_profile(ctx, False)
            r["kernel_ms"] = {k: v[0] / max(1, v[1]) for k, v in prof.items()}
            peak = 157.3 if prec == "mfma_fp32" else 2500.0 / 3.0   # BF16x3: three bf16 products per FLOP
            r["contraction_tflops"] = contraction / (r["kernel_ms"]["strip"] * 1e-3) / 1e12
            r["contraction_peak_tflops"] = peak
            # one captured graph per call: wprep, contraction, fill replayed without host launch work
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                call()
            torch.cuda.current_stream().wait_stream(side)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                call()
            r["graph_ms_per_call"] = _timed(torch, graph.replay, steps, warm)
            del graph
        if check_rows is not None:
            call()
            torch.cuda.synchronize()
            errs = {}
            for m in range(len(lmaxes)):
                K = outs[m][:, torch.as_tensor(check_rows[m].astype(np.int64)).cuda(), :].cpu().numpy()
                Kr, Ar = refs[m]
                for i, s in enumerate(("TT", "TE", "EE", "BB")):
                    nz = Ar[i] > 0
                    e = float(np.max(np.abs(K[i][nz] - Kr[i][nz]) / Ar[i][nz]))
                    errs[s] = max(errs.get(s, 0.0), e)
            r["max_rel_err"] = errs
            r["checked"] = "rows 2, lmax/2, lmax of every mask against the oracle"
        out["batched32_lmax500to4000_" + prec] = r
        print("[bench] batched %s: %.3f ms/call %s" % (prec, ms, r.get("max_rel_err", "")), file=sys.stderr,
              flush=True)
    couple.couple_free(ctx)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=("fp64", "fp32c", "both"))
    ap.add_argument("--lmax", type=int, default=6000)
    ap.add_argument("--cpu-rows", type=int, default=400, help="oracle rows timed for cpu_baseline (0: skip)")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle error check")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the band-limited and batched workload timings reported beside the headline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the coupling path has no multi-GPU form; every work item is "
              "independent, so rows would shard by equal work with one gather of K at the end.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_15605_amd import couple, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    lmax = args.lmax
    spectra = ("TT", "TE", "EE", "BB")
    W = synth.workload_windows(2, lmax=lmax)
    dW = [torch.as_tensor(w).cuda() for w in W]
    ctx = couple.couple_init(lmax)
    out = torch.empty((4, lmax + 1, lmax + 1), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    precisions = ["fp32c", "fp64"] if args.precision == "both" else [args.precision]
    n_el = 4 * (lmax + 1) ** 2
    T = triples(lmax)
    results = {}
    for prec in precisions:
        try:
            couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=prec, out=out, stream=stream)
        except couple.CoupleError as e:
            if e.code == couple.COUPLE_ENOTSUP:
                results[prec] = {"status": "not available: %s" % e}
                continue
            raise
        for _ in range(max(0, args.warmup - 1)):
            couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=prec, out=out, stream=stream)
        torch.cuda.synchronize()
        couple.couple_profile(ctx, True)
        t0 = time.perf_counter()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        ev0.record(stream)
        marks[0].record(stream)
        for i in range(args.steps):
            couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=prec, out=out, stream=stream)
            marks[i + 1].record(stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)])
        prof = couple.couple_profile_read(ctx)
        couple.couple_profile(ctx, False)
        ms_step = ev0.elapsed_time(ev1) / args.steps
        strip_ms, strip_n = prof["strip"]
        strip_avg = strip_ms / max(1, strip_n)
        flops = FLOP_PER_TRIPLE_POL * T
        r = {
            "ms_per_step": ms_step,
            "ms_per_step_std": float(per_step.std(ddof=1)) if args.steps > 1 else 0.0,
            "wall_ms_per_step": 1e3 * wall / args.steps,
            "k_elements_per_s": n_el / (ms_step * 1e-3),
            "kernel_ms": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
            "strip_tflops": flops / (strip_avg * 1e-3) / 1e12,
            "strip_effective_tflops": FLOP_PER_TRIPLE_PAPER * T / (strip_avg * 1e-3) / 1e12,
        }
        r["strip_roofline_frac"] = r["strip_tflops"] / PEAK_VALU_TFLOPS[prec]
        r["strip_effective_frac"] = r["strip_effective_tflops"] / PEAK_VALU_TFLOPS[prec]
        results[prec] = r
        print("[bench] %s: %.3f ms/step, strip %.3f ms, %.2f TFLOP/s alg" %
              (prec, ms_step, strip_avg, r["strip_tflops"]), file=sys.stderr, flush=True)

    # oracle: CPU baseline on a bounded sample of rows, and the error of each path on it
    cpu = None
    if args.cpu_rows > 0:
        from oracle import bulk
        rows = bench_rows(lmax, args.cpu_rows)
        n_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        Kr, Ar = bulk.coupling_rows(lmax, *W, rows=rows, spectra=spectra, n_threads=n_threads)
        dt = time.perf_counter() - t0
        cpu = {"value": len(rows) * (lmax + 1) * 4 / dt, "unit": "K elements/s", "cores": n_threads,
               "kind": "oracle",
               "sample": "%d seeded rows of %d (all 4 spectra, all l2) at lmax=%d: %.1f s on %d threads of %s"
                         % (len(rows), lmax + 1, lmax, dt, n_threads, cpu_model())}
        if not args.no_check:
            rows_t = torch.as_tensor(rows.astype(np.int64)).cuda()
            for prec in precisions:
                if "ms_per_step" not in results[prec]:
                    continue
                couple.couple_matrix(ctx, *dW, lmax, spectra=spectra, precision=prec, out=out, stream=stream)
                torch.cuda.synchronize()
                K = out[:, rows_t, :].cpu().numpy()
                errs = {}
                for i, s in enumerate(spectra):
                    nz = Ar[i] > 0
                    errs[s] = float(np.max(np.abs(K[i][nz] - Kr[i][nz]) / Ar[i][nz]))
                    assert np.all(K[i][~nz] == 0.0)
                results[prec]["max_rel_err"] = errs
                results[prec]["max_rel_err_te_plain"] = te_plain_error(K[1], Kr[1], Ar[1])

    extras = {} if args.no_extras else run_extras(torch, couple, synth, args)
    if not args.no_extras:
        extras.update(run_context(torch, couple, synth))
        extras["scaling_lmax500to6000"] = run_scaling(torch, couple, synth)

    head = "fp32c" if "ms_per_step" in results.get("fp32c", {}) else "fp64"
    h = results[head]
    strip_avg = h["kernel_ms"]["strip"]
    achieved = FLOP_PER_TRIPLE_POL * T / (strip_avg * 1e-3) / 1e12
    line = {
        "metric": "K elements/s at lmax=6000 TT+pol, FP32-comp/MFMA vs FP64 plain, max rel err",
        "value": h["k_elements_per_s"],
        "unit": "K elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "ms_per_step_std": h["ms_per_step_std"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32c" else "f64",
        "data": "synthetic",
        "config": {"workload": "pol4_lmax6000: TT,TE,EE,BB at lmax=6000, one synthetic window "
                               "(W_0=4pi*0.4, (l+1)^-2 exp(-(l/1500)^2) lognormal 0.1, seeds 2000/2001/2002)",
                   "lmax": lmax, "spectra": list(spectra), "precision": head,
                   "triples": T, "elements_per_step": n_el},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS[head], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS[head],
                     "traffic": measured_traffic("strip_%s_kernel" % head),
                     "kernel": "strip_%s_kernel (l3 reduction)" % head, "flop_per_triple": FLOP_PER_TRIPLE_POL,
                     "effective": {"flop_per_triple": FLOP_PER_TRIPLE_PAPER,
                                   "achieved": FLOP_PER_TRIPLE_PAPER * T / (strip_avg * 1e-3) / 1e12,
                                   "frac": FLOP_PER_TRIPLE_PAPER * T / (strip_avg * 1e-3) / 1e12
                                   / PEAK_VALU_TFLOPS[head],
                                   "note": "the method's count with X^2 formed per triple (3 multiplies)"},
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated; "
                                     "profiles/strip_pol4_lmax6000_traffic.md)"},
        "cpu_baseline": cpu,
        "precisions": results,
        "other_workloads": extras,
    }
    print(json.dumps(line), flush=True)
    couple.couple_free(ctx)


if __name__ == "__main__":
    main()
