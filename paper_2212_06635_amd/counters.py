"""Summaries of rocprofv3 runs for the stencil kernels, and the per-launch HBM
traffic they record.

A summary is made from three runs of the same program (``bench.py --mode
kernels``, which ends with device copies of a 2 GiB buffer), after one run
that tunes the launch shapes into a cache file, so that the profiled runs
launch what the benchmark launches without the tuner's sweeps:

    TMX_TUNE_CACHE=D/tune.txt python3 bench.py --mode kernels
    TMX_TUNE_CACHE=D/tune.txt rocprofv3 --kernel-trace --stats --output-format csv -d D/p_k -o k -- python3 bench.py --mode kernels --no-tune
    TMX_TUNE_CACHE=D/tune.txt rocprofv3 --pmc FETCH_SIZE --output-format csv -d D/p_f -o f -- python3 bench.py --mode kernels --no-tune
    TMX_TUNE_CACHE=D/tune.txt rocprofv3 --pmc WRITE_SIZE --output-format csv -d D/p_w -o w -- python3 bench.py --mode kernels --no-tune
    python3 -m paper_2212_06635_amd.counters stencil D out.txt

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read for
the plain copy of known size.  The summary carries a digest of the kernel
sources, so that a reader (bench.py) uses its traffic figures only while the
kernels are the ones that were measured.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STENCIL_SOURCES = ("csrc/dslash.hip", "csrc/tmx_device.h", "csrc/tmx_kernels.h")
COPY_BYTES = 2 ** 31

# rocprof kernel name -> bench label; dslash_kernel<P, NF, MODE, SPT> (sites per
# thread: the tuned launch of a kernel uses one of the two)
LABELS = {f"void tmx::dslash_kernel<{p}, 1, {m}, {t}>(tmx::DslashArgs)": f"K{m + 1}_{n}"
          for p, n in ((0, "f64"), (1, "f32"), (2, "f16")) for m in (0, 1) for t in (1, 2)}


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in STENCIL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_bytes_per_site(kernel: str) -> float:
    """Algorithmic bytes per output site of one stencil launch (each input read
    once): links (2 rows), blocks, spinors; FP16 adds a 4-byte scale per
    spinor read or written."""
    prec = "f64" if "f64" in kernel else ("f32" if "f32" in kernel else "f16")
    b = {"f64": 8, "f32": 4, "f16": 2}[prec]
    nd = "_nd" in kernel
    nrhs = int(kernel.split("_r")[-1]) if "_r" in kernel else 1
    nf = 2 if nd else 1
    norm = 4 if prec == "f16" else 0
    if kernel.startswith("K1"):
        fixed = 96 * b + (144 * b)  # 8 links x 12 reals; inverse blocks (deg: 2 full 6x6; nd: A + B Hermitian)
        spin = nf * (48 * b + 2 * norm)  # read in, write out
    else:
        fixed = 96 * b + 72 * b  # links; Hermitian A_oo
        spin = nf * (72 * b + 3 * norm)  # read hop input and x, write out
    return fixed + nrhs * spin


def _stats(path):
    out = {}
    for r in csv.DictReader(open(path)):
        out[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]))
    return out


def _pmc(path, counter):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def _copy_kib(path, counter):
    """Counter value (KiB) of the 2 GiB calibration copies: the median of the
    three largest copy dispatches (smaller copies in the same run are not
    the calibration)."""
    vals = sorted(float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                  if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"])
    top = vals[-3:]
    return top[len(top) // 2]


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def summarize(d: str, vh: int) -> str:
    st = _stats(_find(os.path.join(d, "p_k"), "kernel_stats.csv"))
    pf = _find(os.path.join(d, "p_f"), "counter_collection.csv")
    pw = _find(os.path.join(d, "p_w"), "counter_collection.csv")
    f, w = _pmc(pf, "FETCH_SIZE"), _pmc(pw, "WRITE_SIZE")
    copy_f, copy_w = _copy_kib(pf, "FETCH_SIZE"), _copy_kib(pw, "WRITE_SIZE")
    sf, sw = COPY_BYTES / 1024 / copy_f, COPY_BYTES / 1024 / copy_w
    copy_ns = next(v for k, v in st.items() if "copyBuffer" in k)[1]
    lines = [
        f"# Schur-operator stencil kernels, V/2 = {vh} sites per launch, MI355X",
        "# commands (from /tmp, TMPDIR=/tmp; <repo> = repository root; the first run tunes the launch shapes",
        "#   into the cache the profiled runs read, so they launch what the benchmark launches):",
        "#   TMX_TUNE_CACHE=<dir>/tune.txt python3 <repo>/bench.py --mode kernels",
        "#   TMX_TUNE_CACHE=<dir>/tune.txt rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/p_k -o k -- python3 <repo>/bench.py --mode kernels --no-tune",
        "#   TMX_TUNE_CACHE=<dir>/tune.txt rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/p_f -o f -- python3 <repo>/bench.py --mode kernels --no-tune",
        "#   TMX_TUNE_CACHE=<dir>/tune.txt rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/p_w -o w -- python3 <repo>/bench.py --mode kernels --no-tune",
        "#   python3 -m paper_2212_06635_amd.counters stencil <dir> <this file>",
        "# bench.py --mode kernels: 10 Mhat applications per precision on the 32^3x64 field (eps 0.25, seed 4),",
        "#   then 3 device copies of a 2 GiB buffer",
        f"# counter calibration on the 2 GiB copy: FETCH_SIZE {copy_f:.1f} KiB, WRITE_SIZE {copy_w:.1f} KiB per dispatch",
        f"#   -> FETCH scale {sf:.3f}, WRITE scale {sw:.3f} (applied below)",
        f"# stencil sources digest: {source_digest()}",
        "",
        f"{'kernel':8s} {'calls':>5s} {'avg_us':>8s} {'alg_MB':>8s} {'alg_GB/s':>9s} {'%8TB/s':>7s} "
        f"{'fetch_MB':>9s} {'write_MB':>9s} {'fetch/alg':>9s} {'traffic_GB/s':>12s}",
    ]
    for kname, lab in LABELS.items():
        if kname not in st:
            continue
        calls, avg = st[kname]
        alg = kernel_bytes_per_site(lab) * vh
        fe = f[kname] * 1024 * sf
        wr = w[kname] * 1024 * sw
        rd = alg - (24 * {"f64": 8, "f32": 4, "f16": 2}[lab[3:]] + (4 if "f16" in lab else 0)) * vh
        lines.append(f"{lab:8s} {calls:5d} {avg / 1e3:8.1f} {alg / 1e6:8.1f} {alg / (avg * 1e-9) / 1e9:9.1f} "
                     f"{100 * alg / (avg * 1e-9) / 8e12:7.1f} {fe / 1e6:9.1f} {wr / 1e6:9.1f} {fe / rd:9.3f} "
                     f"{(fe + wr) / (avg * 1e-9) / 1e9:12.1f}")
    lines.append("")
    lines.append(f"copy 2 GiB: {copy_ns / 1e3:.1f} us avg -> {2 * COPY_BYTES / (copy_ns * 1e-9) / 1e9:.1f} GB/s read+write")
    return "\n".join(lines) + "\n"


def read_traffic(path: str, label: str):
    """HBM bytes per launch of kernel `label` (FETCH + WRITE, scaled) from a
    summary, or None when the file is absent, lacks the kernel, or was taken
    from other kernel sources than the current ones."""
    try:
        text = open(path).read().splitlines()
    except OSError:
        return None
    digest = None
    for ln in text:
        if ln.startswith("# stencil sources digest:"):
            digest = ln.split(":", 1)[1].strip()
    if digest != source_digest():
        return None
    for ln in text:
        p = ln.split()
        if p and p[0] == label and len(p) >= 8:
            return (float(p[6]) + float(p[7])) * 1e6
    return None


def kernel_table(stats_csv: str, title: str, command: str) -> str:
    """Per-kernel time table of one rocprofv3 --kernel-trace --stats run."""
    rows = []
    for r in csv.DictReader(open(stats_csv)):
        rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["TotalDurationNs"]),
                     float(r["Percentage"])))
    rows.sort(key=lambda t: -t[3])
    lines = [f"# {title}", f"# command: {command}", "",
             f"{'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'%':>6s}  kernel"]
    for name, calls, avg, tot, pct in rows:
        short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"{calls:6d} {avg / 1e3:10.1f} {tot / 1e6:10.2f} {pct:6.2f}  {short}")
    return "\n".join(lines) + "\n"


def network(d: str, v: int) -> str:
    """Network layer kernels: time, counter traffic and matrix-core rate."""
    st = _stats(_find(os.path.join(d, "p_k"), "kernel_stats.csv"))
    pf = _find(os.path.join(d, "p_f"), "counter_collection.csv")
    pw = _find(os.path.join(d, "p_w"), "counter_collection.csv")
    f, w = _pmc(pf, "FETCH_SIZE"), _pmc(pw, "WRITE_SIZE")
    copy_f, copy_w = _copy_kib(pf, "FETCH_SIZE"), _copy_kib(pw, "WRITE_SIZE")
    sf, sw = COPY_BYTES / 1024 / copy_f, COPY_BYTES / 1024 / copy_w
    lines = [
        f"# learned-preconditioner layer kernels, V = {v} sites, MI355X",
        "# commands (from /tmp, TMPDIR=/tmp; <repo> = repository root):",
        "#   rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/p_k -o k -- python3 <repo>/bench.py --mode nn --no-tune",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/p_f -o f -- python3 <repo>/bench.py --mode nn --no-tune",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/p_w -o w -- python3 <repo>/bench.py --mode nn --no-tune",
        "#   python3 -m paper_2212_06635_amd.counters network <dir> <this file>",
        "# bench.py --mode nn: 5 applications of K (layers 1->8, 8->8, 8->8, 8->1) on the 32^3x64 field",
        "#   (the one-channel layers 1->8 and 8->1 on the vector ALUs, the 8->8 layers on the matrix cores),",
        "#   then 5 of P_1 = L_1^dagger L_1 through path channels (P1_UP: 1->8 on even tiles, P1_DN),",
        "#   then 3 device copies of a 2 GiB buffer (counter calibration)",
        f"# FETCH scale {sf:.3f}, WRITE scale {sw:.3f}; 8->8 layer work per site: dense 2 x 64 x 64 x 27 flops",
        "#   (9 paths x 3 colours of the real 64 x 64 Kronecker product the matrix cores run, TF_dense) and the",
        "#   method's factorised count 82944 flops (C_d (x) Gamma_d applied as two small products, TF_method)",
        "",
        f"{'kernel':10s} {'calls':>5s} {'avg_us':>8s} {'fetch_MB':>9s} {'write_MB':>9s} {'GB/s':>7s} {'TF_dense':>8s} {'TF_method':>9s}",
    ]
    for name, (calls, avg) in sorted(st.items()):
        if "nn_layer_kernel" in name:
            tag = name[name.index("<") + 1:name.index(">")].replace(", ", "x")
        elif "nn_up_kernel" in name:
            # one-channel layer on the vector ALUs (forward 1->8, adjoint of 8->1), per source precision;
            # on even tiles only: the first half of P_1 (path channels)
            targs = name[name.index("<") + 1:name.index(">")].split(", ") if "<" in name else ["", "false"]
            tag = ("P1_UP" if targs[-1] == "true" else "1x8") + "_" + targs[0]
        elif "nn_p1_down_kernel" in name:
            tag = "P1_DN_" + name[name.index("<") + 1:name.index(">")] if "<" in name else "P1_DN"
        elif "nn_down_kernel" in name:
            tag = "8x1"     # forward 8->1, adjoint of 1->8
        else:
            continue
        fe = f.get(name, 0.0) * 1024 * sf
        wr = w.get(name, 0.0) * 1024 * sw
        tf = 2 * 64 * 64 * 27 * v / (avg * 1e-9) / 1e12 if tag == "8x8" else float("nan")
        tm = 82944 * v / (avg * 1e-9) / 1e12 if tag == "8x8" else float("nan")
        lines.append(f"NN_{tag:7s} {calls:5d} {avg / 1e3:8.1f} {fe / 1e6:9.1f} {wr / 1e6:9.1f} "
                     f"{(fe + wr) / (avg * 1e-9) / 1e9:7.1f} {tf:8.1f} {tm:9.1f}")
    return "\n".join(lines) + "\n"


# force kernels: (kernel-name fragment, label, model bytes per site, read, write)
FORCE_KERNELS = (
    ("hop_force_kernel", "HOP_FORCE", 1344, 768, 576),          # a, b 2 x 192, 4 links x 96 | 4 outputs x 144
    ("clover_insertion_kernel", "CLOV_INSERT", 816, 384, 432),   # a, b | 6 Hermitian planes x 72
    # 4 links x 96, 6 insertion planes x 72 | 6 plaquettes x 128 (traceless K, A)
    ("clover_loop_kernel", "CLOV_LOOPS", 1584, 816, 768),
    # 6 plaquettes x 128, 6 insertion planes x 72, 4 links x 96 | 4 outputs x 144
    ("clover_link_kernel", "CLOV_LINKS", 2160, 1584, 576),
)


def force(d: str, v: int) -> str:
    """Force kernels: time, counter traffic against the byte model of each."""
    st = _stats(_find(os.path.join(d, "p_k"), "kernel_stats.csv"))
    pf = _find(os.path.join(d, "p_f"), "counter_collection.csv")
    pw = _find(os.path.join(d, "p_w"), "counter_collection.csv")
    f, w = _pmc(pf, "FETCH_SIZE"), _pmc(pw, "WRITE_SIZE")
    copy_f, copy_w = _copy_kib(pf, "FETCH_SIZE"), _copy_kib(pw, "WRITE_SIZE")
    sf, sw = COPY_BYTES / 1024 / copy_f, COPY_BYTES / 1024 / copy_w
    lines = [
        f"# fermion-force kernels (hopping term; clover term = insertions + plaquette loops + link sums), V = {v} sites "
        "(all 4V links), MI355X",
        "# commands (from /tmp, TMPDIR=/tmp; <repo> = repository root):",
        "#   rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/p_k -o k -- python3 <repo>/bench.py --mode force --no-tune",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/p_f -o f -- python3 <repo>/bench.py --mode force --no-tune",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/p_w -o w -- python3 <repo>/bench.py --mode force --no-tune",
        "#   python3 -m paper_2212_06635_amd.counters force <dir> <this file>",
        "# bench.py --mode force: 10 hopping-force and 10 clover-force calls on the 32^3x64 field, "
        "then 3 device copies of 2 GiB",
        f"# FETCH scale {sf:.3f}, WRITE scale {sw:.3f}; model bytes per site: "
        + ", ".join(f"{lab} {b} (read {r}, write {wr})" for _, lab, b, r, wr in FORCE_KERNELS),
        "",
        f"{'kernel':12s} {'calls':>5s} {'avg_us':>8s} {'model_MB':>9s} {'fetch_MB':>9s} {'write_MB':>9s} {'model_GB/s':>10s} {'%8TB/s':>7s}",
    ]
    for frag, label, bps, _, _ in FORCE_KERNELS:
        for name, (calls, avg) in sorted(st.items()):
            if frag not in name:
                continue
            model = float(bps) * v
            fe = f.get(name, 0.0) * 1024 * sf
            wr = w.get(name, 0.0) * 1024 * sw
            gbs = model / (avg * 1e-9) / 1e9
            lines.append(f"{label:12s} {calls:5d} {avg / 1e3:8.1f} {model / 1e6:9.1f} {fe / 1e6:9.1f} {wr / 1e6:9.1f} "
                         f"{gbs:10.1f} {gbs / 80:7.1f}")
    return "\n".join(lines) + "\n"


SQ_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU",
               "SQ_ACTIVE_INST_VMEM", "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD")


def sq_table(dirs) -> str:
    """Wave-level counters of the hot kernels from one --pmc pass per program
    (`dirs`: label=directory pairs): the share of each wave's life spent
    waiting on an operand (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) and issuing
    vector ALU work (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES), and the VALU and
    vector-memory-read instructions per wave."""
    lines = [
        "# wave-level SQ counters of the hot kernels, 32^3x64, MI355X",
        "# commands (from /tmp, TMPDIR=/tmp; <repo> = repository root), one per bench mode m in nn, force, kernels:",
        "#   rocprofv3 --pmc " + " ".join(SQ_COUNTERS) + " --output-format csv -d <dir>/sq_m -o q -- "
        "python3 <repo>/bench.py --mode m --no-tune",
        "#   python3 -m paper_2212_06635_amd.counters sq nn=<dir>/sq_nn force=<dir>/sq_force "
        "kernels=<dir>/sq_kernels <this file>",
        "# wait = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES, valu = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES (per wave, summed",
        "#   over the dispatches of a kernel); insts per wave = SQ_INSTS_* / SQ_WAVES",
        "",
        f"{'mode':8s} {'kernel':44s} {'disp':>4s} {'waves/disp':>10s} {'wait':>5s} {'valu':>5s} "
        f"{'valu/wave':>9s} {'vmem_rd/wave':>12s}",
    ]
    for item in dirs:
        label, d = item.split("=", 1)
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
            agg[r["Kernel_Name"]][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[r["Kernel_Name"]].add(r.get("Dispatch_Id", ""))
        for name in sorted(agg):
            short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
            if not any(t in short for t in ("dslash_kernel", "nn_", "force_kernel", "insertion_kernel", "loop_kernel",
                                            "link_kernel")):
                continue
            if "build" in short or "links" in short:
                continue
            v, n = agg[name], max(len(disp[name]), 1)
            wc = max(v["SQ_WAVE_CYCLES"], 1.0)
            nw = max(v["SQ_WAVES"], 1.0)
            lines.append(f"{label:8s} {short[:44]:44s} {n:4d} {nw / n:10.0f} {v['SQ_WAIT_INST_ANY'] / wc:5.2f} "
                         f"{v['SQ_ACTIVE_INST_VALU'] / wc:5.2f} {v['SQ_INSTS_VALU'] / nw:9.0f} "
                         f"{v['SQ_INSTS_VMEM_RD'] / nw:12.0f}")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    usage = ("usage: python3 -m paper_2212_06635_amd.counters stencil <rocprof dir> <summary>\n"
             "       python3 -m paper_2212_06635_amd.counters network <rocprof dir> <summary>\n"
             "       python3 -m paper_2212_06635_amd.counters force <rocprof dir> <summary>\n"
             "       python3 -m paper_2212_06635_amd.counters stats <kernel_stats.csv> <summary> <title> <command>\n"
             "       python3 -m paper_2212_06635_amd.counters sq <label>=<rocprof dir> ... <summary>")
    a = sys.argv[1:]
    if len(a) >= 3 and a[0] == "stencil":
        txt = summarize(a[1], 1048576)
    elif len(a) >= 3 and a[0] == "network":
        txt = network(a[1], 2097152)
    elif len(a) >= 3 and a[0] == "force":
        txt = force(a[1], 2097152)
    elif len(a) >= 3 and a[0] == "sq":
        txt = sq_table(a[1:-1])
    elif len(a) == 5 and a[0] == "stats":
        txt = kernel_table(a[1], a[3], a[4])
    else:
        print(usage, file=sys.stderr)
        sys.exit(2)
    with open(a[-1] if a[0] == "sq" else a[2], "w") as fh:
        fh.write(txt)
    print(txt, end="")
