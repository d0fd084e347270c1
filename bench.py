"""Throughput of the local SpMM hot path on one MI355X, as one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step is one pass of the hot path over one batch of synthetic input that is
already resident in HBM.  The default workload is the forward and backward of one
GNN-shaped layer: a 2,097,152^2 sparse A with heavy-tailed row degrees (Pareto(2.1)
with mean 32 and longest row 65,536, uniform distinct columns, values N(0,1)/sqrt(deg)),
dense B and dC of 2,097,152 x 128 FP32 N(0,1): C = A B, dA = the sampled dense-dense
product on A's pattern, dB = A^T dC (three passes of 2 nnz N flops).  The same step with
B, C, dC and dB in BF16 is reported beside it, and the error of every result against
the FP64 oracle on a sample.  Other workloads:

    rmat22_rowblock0_4x4_n128  one GPU's share of a 4 x 4 stationary-C SpMM (Algorithm 2):
                            row block 0 of an R-MAT scale-22, edge-factor-16 matrix (Graph500
                            quadrant probabilities, duplicates merged, U[-1,1) FP32 values) times
                            B_k of 1,048,576 x 128 FP32 over its 4 k-tiles, C written once
    er4096_n32              4096^2 uniform tile, 16 non-zeros per row, N = 32, forward
    powerlaw2m_n128_fwdbwd  2,097,152^2 heavy-tailed rows (mean 32, max 65,536), N = 128,
                            forward + dA (sampled dense-dense product) + dB = A^T dC
    powerlaw2m_n128_fwdbwd_bf16  the same with B, C, dC and dB in BF16 (FP32 accumulation)
    powerlaw2m_n512_fwdbwd  the same matrix at N = 512 (library default shapes: the fused
                            backward in column windows)
    rmat23_n256_bf16        R-MAT scale 23, edge factor 32, N = 256, BF16 B and C
    rmat23_n256_f32         the same with FP32 B and C
    stationary_a_rmat22_tile00_n128x4
                            stationary-A local step: partial products of R-MAT tile (0,0) with 4
                            column blocks of N = 128, each added into its C tile
    stationary_a_rmat22_rowblock0_4x4_grid
                            stationary-A step of a row block with work stealing: the 16 products
                            A(0,k) B(k,j) handed out through a 3-D reservation grid, partials drained
                            in k order; the 2-D grid, no stealing, no grid and a launch per product
                            are reported beside it
    spgemm_rmat18_ef16_aa   local SpGEMM C = A A, R-MAT scale 18, edge factor 16 (numeric phase;
                            the symbolic phase is reported beside it)
    spgemm_er1m16_aa        local SpGEMM C = A A, 1,048,576^2 uniform, 16 per row
    uneven512_batched       512 uneven tiles (rows 1,024..65,536, 4..256 non-zeros per row,
                            N_t in {32..256}) in one batched launch (one kernel for every item
                            class, persistent claiming), per-tile autotuned variants; the
                            per-tile launch loop and the other launch forms are reported beside it
    gather_<w>b_4096mib     gather probe over a 4 GiB table (w = 512, 128, 16 bytes per row): a
                            kernel of known bytes for calibrating the HBM counters
    copy_1gib               a plain 1 GiB device copy, the same for streaming traffic

value = 2 * nnz * N * passes / step time (GFLOP/s).  The roofline object prices
the step's kernels with their algorithmic bytes (CSR arrays + dense inputs read
once + outputs written once; the performance-model accounting of Section 4)
against the 8 TB/s HBM peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HANDLE_OPTS = {}
AUTOTUNE = False

# Kernel variant (kind, lanes, vec) and split-row plan (long_row, segment) of each
# single-tile workload: what spmm_tile_autotune(tune_plan=1) picks for it on MI355X
# (and for the backward's dB pass, what spmm_tile_autotune_bwd picks).
# Pinned, so that a profiled run launches exactly the kernels the timed run launches
# (no autotuner trials); --autotune re-tunes in set-up instead.
PINNED = {
    "rmat22_rowblock0_4x4_n128": {"variant": ("stream", 64, 2), "long_row": 128, "segment": 64},
    "powerlaw2m_n128_fwdbwd": {"variant": ("rowsplit", 64, 1), "long_row": 1024, "segment": 512,
                               "bwd_variant": ("fused", 32, 4, 4)},
    "powerlaw2m_n128_fwdbwd_bf16": {"variant": ("rowsplit", 64, 2), "long_row": 512, "segment": 256,
                                    "bwd_variant": ("fused", 16, 8, 2)},
    "rmat23_n256_bf16": {"variant": ("rowsplit", 64, 4), "long_row": 128, "segment": 64},
    "rmat23_n256_f32": {"variant": ("stream", 64, 2), "long_row": 128, "segment": 64},
}


def _handle_opts(name):
    """Split-row plan for a handle: the command line's, else the workload's pinned one."""
    pin = PINNED.get(name, {})
    out = {}
    for key in ("long_row", "segment"):
        out[key] = HANDLE_OPTS.get(key) or (0 if AUTOTUNE else pin.get(key, 0))
    return out


def _apply_pin(name, tile, N, dtype):
    from paper_2311_18141_amd import ops
    pin = PINNED.get(name)
    if pin is None:
        return None
    kind, lanes, vec = pin["variant"]
    ops.spmm_tile_set_variant(tile, N, dtype, kind, lanes, vec)
    return {"kind": kind, "lanes": lanes, "vec": vec, "pinned": True}


def _library_fwd(N, dtype, rows, empty):
    """The forward kernel (kind, vec) spmm_fwd takes at width N without a variant entry (16-byte
    aligned operands), by the dtype and the tile's share of empty rows (many: more than 1/8).
    FP32: stream kernel on tiles with many empty rows, else row-split, over 64-column windows, or
    128-column ones for N >= 256 and, with many empty rows, for N a multiple of 128.  BF16:
    row-split over the fewest windows of at most 256 columns on the narrowest vector giving that
    count (stream at N = 64 with many empty rows)."""
    e = 4 if dtype == "f32" else 2
    V = 16 // e
    while V > 1 and N % V:
        V //= 2
    sparse = empty * 8 > rows
    if N >= 64 and dtype == "bf16":
        windows = -(-N // 256)
        vb = 1
        while vb * 2 <= V and -(-N // (64 * vb)) > windows:
            vb *= 2
        return ("stream", 1) if vb == 1 and sparse else ("rowsplit", vb)
    if N >= 256 and V >= 2:
        return ("stream" if sparse else "rowsplit", 2)
    if N >= 64:
        return ("stream", 2 if V >= 2 and N % 128 == 0 else 1) if sparse else ("rowsplit", 1)
    return ("rowsplit", V)


def _fwd_variant_or_rule(variant, tile, N, dtype):
    """The forward variant a handle runs at width N: its pinned or tuned entry, else the rule's."""
    if variant is not None:
        return variant
    st = tile.stats()
    kind, vec = _library_fwd(N, dtype, st["rows"], st["empty_rows"])
    return {"kind": kind, "vec": vec, "library_rule": True}


def _library_bwd_fused(N, dtype):
    """Whether spmm_bwd takes the fused form at width N without a variant entry (16-byte aligned
    operands): the widest vector dividing N and 64-lane groups need at most min(8, max(1,
    ceil(N / 256))) column windows."""
    e = 4 if dtype == "f32" else 2
    V = 16 // e
    while V > 1 and N % V:
        V //= 2
    G = 4
    while G < 64 and G * V < N:
        G *= 2
    return -(-N // (G * V)) <= min(8, max(1, -(-N // 256)))


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# Sources of the kernels a workload launches (forward, split-row fix-up, hot-row staging; for the
# backward also SDDMM and value gather; the SpGEMM numeric kernels): a stored counter reading is
# valid while these are unchanged.
FWD_SOURCES = ("elem.hpp", "fwd_common.hpp", "fwd.hip", "hot.hip")
KERNEL_SOURCES = {"powerlaw2m_n128_fwdbwd": FWD_SOURCES + ("bwd.hip",),
                  "powerlaw2m_n128_fwdbwd_bf16": FWD_SOURCES + ("bwd.hip",),
                  "powerlaw2m_n512_fwdbwd": FWD_SOURCES + ("bwd.hip",),
                  "uneven512_batched": ("elem.hpp", "fwd_common.hpp", "batch.hip"),
                  "spgemm_rmat18_ef16_aa": ("spgemm.hip",),
                  "spgemm_er1m16_aa": ("spgemm.hip",)}


def kernel_source_digest(workload: str = "") -> str:
    """SHA-256 over the sources of the kernels `workload` launches (the forward's by default)
    and over its pinned kernel shapes, so that a stored reading lapses when either changes."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2311_18141_amd", "csrc")
    for name in KERNEL_SOURCES.get(workload, FWD_SOURCES):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    if workload in PINNED:
        h.update(b"pin\0" + json.dumps(PINNED[workload], sort_keys=True).encode())
    if workload == "powerlaw2m_n128_fwdbwd":  # its line also runs the BF16 workload's pinned kernels
        h.update(b"pin\0" + json.dumps(PINNED[workload + "_bf16"], sort_keys=True).encode())
    return h.hexdigest()


def stored_traffic(workload: str, key: str = "hbm_bytes_per_step"):
    """HBM bytes per step measured by rocprofv3 counters (profiles/traffic_<workload>.md), or None when
    absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.md" % workload)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != kernel_source_digest(workload):
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _threads():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


# ---------------------------------------------------------------------------
METRIC = "SpMM GFLOP/s (2*nnz*N) and % HBM roofline, fwd+bwd, BF16/batched vs FP32"


class Workload:
    name = ""
    dtype = "f32"
    kernel = ""
    metric = METRIC

    def setup(self):  # build device inputs and handles
        raise NotImplementedError

    def step(self):  # one pass of the hot path (asynchronous)
        raise NotImplementedError

    flops = 0.0
    alg_bytes = 0.0
    config = {}

    def cpu_sample(self):  # -> (flops, seconds, description)
        raise NotImplementedError

    def extra(self, kernel_ms):  # further objects for the JSON line, given the per-step kernel time
        return {}


REL_DEFINITION = ("rel = |x - x64| / max(|x64|, 2^-20 S); rel_to_scale = |x - x64| / S, S = sum |a||b|; x64 = the "
                  "FP64 oracle on the FP32 operands (total error) or on their BF16 roundings (the kernels' own error)")


def _err_stats(got, ref, S):
    """Max / mean relative error of one sampled result against the oracle."""
    from oracle import compare
    g = got.float().cpu().numpy().astype(np.float64)
    rel = compare.relative_stats(g, ref, S)
    sc = compare.fp32_stats(g, ref, S)
    return {"max_rel": float("%.4g" % rel["max_rel"]), "mean_rel": float("%.4g" % rel["mean_rel"]),
            "max_rel_to_scale": float("%.4g" % sc["max_rel_to_scale"]),
            "mean_rel_to_scale": float("%.4g" % sc["mean_rel_to_scale"]),
            "nonfinite": rel["nonfinite"], "entries": int(g.size)}


def _fwd_bytes(tiles, N, esize):
    b = 0
    for t in tiles:
        b += 8 * t.nnz + 4 * (t.rows + 1) + t.cols * N * esize
    return b + tiles[0].rows * N * esize


class TileRowForward(Workload):
    """C = sum_k A_k B_k over a tile row (one tile or several k-tiles)."""

    def __init__(self, name, make_tiles, N, dtype, config):
        self.name = name
        self.make_tiles = make_tiles
        self.N = N
        self.dtype = dtype
        self.config = config
        self.kernel = "spmm_fwd (fwd_main + fwd_fixup)"

    def setup(self):
        import torch
        import synth
        from paper_2311_18141_amd import ops
        t0 = time.time()
        self.tiles = self.make_tiles()
        _log("%s: inputs generated in %.1f s (nnz %d)" % (self.name, time.time() - t0, sum(t.nnz for t in self.tiles)))
        rng = synth.streams(self.config.get("seed", 1))[2]
        self.Bh = [synth.dense(t.cols, self.N, rng) for t in self.tiles]
        tdt = torch.float32 if self.dtype == "f32" else torch.bfloat16
        dev = "cuda:0"
        self.dev_tiles = [(torch.from_numpy(t.rowptr).to(dev), torch.from_numpy(t.colind).to(dev),
                           torch.from_numpy(t.values).to(dev), t.cols) for t in self.tiles]
        self.B = [torch.from_numpy(b).to(tdt).to(dev) for b in self.Bh]
        self.tile = ops.spmm_tile_create(self.tiles[0].rows, self.dev_tiles, validate=True,
                                         **_handle_opts(self.name))
        self.C = torch.empty(self.tiles[0].rows, self.N, dtype=tdt, device=dev)
        if AUTOTUNE:
            t0 = time.time()
            chosen = ops.spmm_tile_autotune(self.tile, self.B, self.C, tune_plan=True)
            _log("%s: autotuned in %.1f s: %s" % (self.name, time.time() - t0, chosen))
            self.config["variant"] = chosen
        else:
            self.config["variant"] = _apply_pin(self.name, self.tile, self.N, tdt)
        self.config["variant"] = _fwd_variant_or_rule(self.config["variant"], self.tile, self.N, self.dtype)
        fk = "fwd_stream" if self.config["variant"]["kind"] == "stream" else "fwd_main"
        hs = "hot_stage + " if self.tile.stats()["hot_rows"] > 0 else ""
        self.kernel = "spmm_fwd (%s%s + fwd_fixup)" % (hs, fk)
        self.ws = self.tile.workspace(self.N)
        nnz = sum(t.nnz for t in self.tiles)
        self.flops = 2.0 * nnz * self.N
        e = 4 if self.dtype == "f32" else 2
        self.alg_bytes = float(_fwd_bytes(self.tiles, self.N, e))
        # each non-zero gathers its B row (e N bytes) from the k-tiles' B (sum of cols_k x e N bytes)
        self.gather_items = [(float(nnz) * e * self.N, sum(t.cols for t in self.tiles) * e * self.N, e * self.N)]
        self.config = dict(self.config, nnz=nnz, rows=self.tiles[0].rows, N=self.N, k_tiles=len(self.tiles),
                           tile_stats={k: v for k, v in self.tile.stats().items()
                                       if k in ("max_row", "empty_rows", "long_rows", "segments", "long_row",
                                                "segment", "hot_rows", "hot_nnz")})

    def step(self):
        from paper_2311_18141_amd import ops
        ops.spmm_fwd(self.tile, self.B, C=self.C, workspace=self.ws)

    def extra(self, kernel_ms):
        out = {"cache_gather": gather_ceiling_report(self.gather_items, kernel_ms)}
        if self.dtype == "bf16":
            out["f32"] = self._f32_companion(kernel_ms)
        if self.config.get("column_panels"):
            out["column_panels"] = self._column_panels(self.config["column_panels"])
        return out

    def _column_panels(self, counts, steps=5):
        """B-row reuse by column-panel blocking: each k-tile cut into P column panels, one
        forward per panel into the same C (the first writes, the rest accumulate), so that a
        launch gathers only from one panel's B rows (cols / P x N x e bytes, small enough for the
        Infinity Cache) at the price of reading and writing C once per panel instead of once."""
        import torch
        from paper_2311_18141_amd import ops
        e = 4 if self.dtype == "f32" else 2
        dev = self.C.device
        ref = self.C.float()
        out = {"note": "time per step; C equal to the unblocked step's up to summation order "
                       "(max |diff| / max |C|)"}
        for P in counts:
            parts = []
            for t, B in zip(self.tiles, self.B):
                w = -(-t.cols // P)
                rows = np.repeat(np.arange(t.rows, dtype=np.int64), np.diff(t.rowptr))
                pid = t.colind // w
                for p in range(P):
                    sel = pid == p
                    lengths = np.bincount(rows[sel], minlength=t.rows)
                    rp = np.zeros(t.rows + 1, dtype=np.int64)
                    np.cumsum(lengths, out=rp[1:])
                    c0, c1 = p * w, min(t.cols, (p + 1) * w)
                    d = (torch.from_numpy(rp.astype(t.rowptr.dtype)).to(dev),
                         torch.from_numpy((t.colind[sel] - c0).astype(np.int32)).to(dev),
                         torch.from_numpy(t.values[sel]).to(dev), c1 - c0)
                    h = ops.spmm_tile_create(t.rows, [d], validate=True, **_handle_opts(self.name))
                    _apply_pin(self.name, h, self.N, B.dtype)
                    parts.append((h, B[c0:c1], h.workspace(self.N)))
            C = torch.empty_like(self.C)

            def step():
                for i, (h, Bp, ws) in enumerate(parts):
                    ops.spmm_fwd(h, [Bp], C=C, accumulate=i > 0, workspace=ws)
            for _ in range(2):
                step()
            ms = Batched._time(step, steps)
            torch.cuda.synchronize()
            diff = float((C.float() - ref).abs().max() / ref.abs().max())
            panel_bytes = max(t.cols for t in self.tiles) / P * self.N * e
            out[str(P)] = {"ms_per_step": round(ms, 5), "launches": len(parts),
                           "panel_B_MiB": round(panel_bytes / 2 ** 20, 1),
                           "C_bytes_extra_GB": round((len(parts) - 1) * 2 * self.tiles[0].rows * self.N * e / 1e9, 3),
                           "rel_diff": diff}
            del parts, C
        return out

    def _f32_companion(self, bf16_ms, steps=10):
        """The same forward with FP32 B and C (the draws before rounding) on the same handle."""
        import torch
        from paper_2311_18141_amd import ops
        self.Bf = [torch.from_numpy(b).to(self.B[0].device) for b in self.Bh]
        self.Cf = torch.empty(self.tiles[0].rows, self.N, device=self.B[0].device)
        pin = PINNED.get(self.name.replace("_bf16", "_f32"))
        cfg = None
        if pin and not AUTOTUNE:
            kind, lanes, vec = pin["variant"]
            ops.spmm_tile_set_variant(self.tile, self.N, torch.float32, kind, lanes, vec)
            cfg = {"kind": kind, "lanes": lanes, "vec": vec, "pinned": True}
        ws = self.tile.workspace(self.N)
        step = lambda: ops.spmm_fwd(self.tile, self.Bf, C=self.Cf, workspace=ws)  # noqa: E731
        for _ in range(2):
            step()
        ms = Batched._time(step, steps)
        return {"ms_per_step": round(ms, 5), "value": round(self.flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                "bf16_speedup": round(ms / bf16_ms, 3), "variant": cfg, "steps": steps,
                "note": "same handle and draws as the BF16 step, B and C in FP32"}

    def accuracy(self):
        """Max and mean relative error of C against the FP64 oracle on 2,000 random rows and the
        longest row, after the timed region: against the oracle on the FP32 draws of B (total
        error) and, for BF16 storage, on their BF16 roundings (the kernels' own error)."""
        import torch
        import oracle
        lens = sum(t.row_lengths() for t in self.tiles)
        rng = np.random.Generator(np.random.PCG64(17))
        rows = np.unique(np.concatenate([rng.choice(self.tiles[0].rows, 2000, replace=False),
                                         [int(np.argmax(lens))]]))
        r_t = torch.from_numpy(rows).to(self.C.device)
        csr = [(t.rowptr, t.colind, t.values) for t in self.tiles]
        torch.cuda.synchronize()
        out = {"sample": "%d rows of C" % len(rows), "definition": REL_DEFINITION}
        rC, SC = oracle.spmm(csr, self.Bh, rows=rows)
        if self.dtype == "f32":
            out["f32"] = {"C": _err_stats(self.C[r_t], rC, SC)}
            return out
        Bt = [oracle.bf16_to_f32(oracle.f32_to_bf16(b)) for b in self.Bh]
        rCt, SCt = oracle.spmm(csr, Bt, rows=rows)
        out["bf16_vs_f32_operands"] = {"C": _err_stats(self.C[r_t], rC, SC)}
        out["bf16_vs_bf16_operands"] = {"C": _err_stats(self.C[r_t], rCt, SCt)}
        if hasattr(self, "Cf"):
            out["f32"] = {"C": _err_stats(self.Cf[r_t], rC, SC)}
        return out

    def cpu_sample(self):
        import oracle
        Bs = self.Bh
        if self.dtype == "bf16":
            Bs = [oracle.bf16_to_f32(oracle.f32_to_bf16(b)) for b in Bs]
        rows = self.tiles[0].rows
        lens = sum(t.row_lengths() for t in self.tiles)
        # rows [0, r): enough non-zeros for about 20 GFLOP of oracle work (or the whole tile row)
        target = 2.0e10 / (2.0 * self.N)
        r = int(min(rows, np.searchsorted(np.cumsum(lens), target) + 1))
        sel = np.arange(r, dtype=np.int64)
        t0 = time.perf_counter()
        oracle.spmm([(t.rowptr, t.colind, t.values) for t in self.tiles], Bs, rows=sel, scale=False)
        dt = time.perf_counter() - t0
        nnz = float(lens[:r].sum())
        return 2.0 * nnz * self.N, dt, "oracle FP64 forward on rows [0, %d) of %d (%d non-zeros)" % (r, rows, nnz)


def _fwdbwd_gather_items(A, N, e, fused):
    """Gathers of one forward + backward step at element size e: the forward reads a B row per
    non-zero; the fused backward a dC row per non-zero (the two-pass form: the SDDMM a B row and
    the dB pass a dC row per non-zero); both backward forms read one 4-byte value per non-zero at
    random (timed as a 16-byte row, the probe's smallest, from a table of the values' size)."""
    row = e * N
    items = [(float(A.nnz) * row, A.cols * row, row), (float(A.nnz) * row, A.rows * row, row),
             (float(A.nnz) * 16, 4 * A.nnz, 16)]
    if not fused:
        items.append((float(A.nnz) * row, A.cols * row, row))
    return items


class ForwardBackward(Workload):
    """Forward, dA = SDDMM on A's pattern, dB = A^T dC: three passes of 2 nnz N flops."""

    def __init__(self, name, make_tile, N, config, dtype="f32"):
        self.name = name
        self.make_tile = make_tile
        self.N = N
        self.config = config
        self.dtype = dtype
        self.kernel = "spmm_fwd + spmm_bwd (fwd_stream, fwd_fixup, sddmm_kernel, gather_values)"

    def setup(self):
        import torch
        import synth
        from paper_2311_18141_amd import ops
        t0 = time.time()
        self.A = self.make_tile()
        _log("%s: inputs generated in %.1f s (nnz %d)" % (self.name, time.time() - t0, self.A.nnz))
        rs = synth.streams(self.config.get("seed", 3))
        self.Bh = synth.dense(self.A.cols, self.N, rs[2], "normal")
        self.dCh = synth.dense(self.A.rows, self.N, rs[3], "normal")
        dev = "cuda:0"
        t = (torch.from_numpy(self.A.rowptr).to(dev), torch.from_numpy(self.A.colind).to(dev),
             torch.from_numpy(self.A.values).to(dev), self.A.cols)
        self.tile = ops.spmm_tile_create(self.A.rows, [t], validate=True, transpose=True,
                                         **_handle_opts(self.name))
        tdt = torch.float32 if self.dtype == "f32" else torch.bfloat16
        self.B = torch.from_numpy(self.Bh).to(tdt).to(dev)
        self.dC = torch.from_numpy(self.dCh).to(tdt).to(dev)
        self.C = torch.empty(self.A.rows, self.N, device=dev, dtype=tdt)
        if AUTOTUNE:
            t0 = time.time()
            chosen = ops.spmm_tile_autotune(self.tile, [self.B], self.C, tune_plan=True)
            _log("%s: forward autotuned in %.1f s: %s" % (self.name, time.time() - t0, chosen))
            self.config["variant"] = chosen
        else:
            self.config["variant"] = _apply_pin(self.name, self.tile, self.N, tdt)
        self.dA = torch.empty(self.A.nnz, device=dev)
        self.dB = torch.empty(self.A.cols, self.N, device=dev, dtype=tdt)
        # the dB pass (forward kernels over the transpose) has its own variant
        if AUTOTUNE:
            t0 = time.time()
            chosen = ops.spmm_tile_autotune_bwd(self.tile, self.dC, self.dB, B=self.B, dA=self.dA)
            _log("%s: backward autotuned in %.1f s: %s" % (self.name, time.time() - t0, chosen))
            self.config["bwd_variant"] = chosen
        elif PINNED.get(self.name, {}).get("bwd_variant"):
            kind, lanes, vec, depth = PINNED[self.name]["bwd_variant"]
            ops.spmm_tile_set_bwd_variant(self.tile, self.N, tdt, kind, lanes, vec, depth)
            self.config["bwd_variant"] = {"kind": kind, "lanes": lanes, "vec": vec, "depth": depth, "pinned": True}
        # the SDDMM's shape (lanes x non-zeros per group), pinned like the variants
        sd = PINNED.get(self.name, {}).get("sddmm")
        if sd:
            ops.spmm_tile_set_sddmm_variant(self.tile, self.N, sd[0], sd[1])
            self.config["sddmm"] = {"lanes": sd[0], "nnz_per_group": sd[1], "pinned": True}
        self.config["variant"] = _fwd_variant_or_rule(self.config["variant"], self.tile, self.N, self.dtype)
        fk = "fwd_stream" if self.config["variant"]["kind"] == "stream" else "fwd_main"
        bkind = (self.config.get("bwd_variant") or {}).get("kind")
        if bkind is None:   # no entry: the library's rule, which takes the fused form for these operands
            bkind = "fused" if _library_bwd_fused(self.N, self.dtype) else "stream"
            self.config["bwd_variant"] = {"kind": bkind, "library_rule": True}
        self.fused = bkind == "fused"
        if self.fused:
            self.kernel = "spmm_fwd + spmm_bwd (%s, fwd_fixup, bwd_fused over the transpose)" % fk
        else:
            bk = "fwd_main" if bkind == "rowsplit" else "fwd_stream"
            self.kernel = ("spmm_fwd + spmm_bwd (%s, fwd_fixup, sddmm_kernel, gather_values, %s on the transpose)"
                           % (fk, bk))
        self.wsf = self.tile.workspace(self.N, "fwd")
        self.wsb = self.tile.workspace(self.N, "bwd")
        A, N = self.A, self.N
        e = 4 if self.dtype == "f32" else 2
        self.flops = 3 * 2.0 * A.nnz * N
        fwd = 8 * A.nnz + 4 * (A.rows + 1) + e * A.cols * N + e * A.rows * N
        sddmm = 4 * A.nnz + 4 * (A.rows + 1) + e * A.rows * N + e * A.cols * N + 4 * A.nnz
        dB = 4 * (A.cols + 1) + 12 * A.nnz + e * A.rows * N + e * A.cols * N
        self.alg_bytes = float(fwd + sddmm + dB)
        self.gather_items = _fwdbwd_gather_items(A, N, e, self.fused)
        st = self.tile.stats()
        self.config = dict(self.config, nnz=A.nnz, rows=A.rows, N=N,
                           tile_stats={k: st[k] for k in ("max_row", "empty_rows", "long_rows", "segments",
                                                          "long_rows_t", "segments_t", "long_row", "segment",
                                                          "hot_rows", "hot_nnz")})

    def step(self):
        from paper_2311_18141_amd import ops
        ops.spmm_fwd(self.tile, [self.B], C=self.C, workspace=self.wsf)
        ops.spmm_bwd(self.tile, self.dC, self.B, dA=self.dA, dB=self.dB, workspace=self.wsb)

    def _pass_ms(self, B, C, dC, dA, dB, reps=10):
        """Mean time of the forward call and of the backward call, each timed on its own."""
        from paper_2311_18141_amd import ops
        f = Batched._time(lambda: ops.spmm_fwd(self.tile, [B], C=C, workspace=self.wsf), reps)
        b = Batched._time(lambda: ops.spmm_bwd(self.tile, dC, B, dA=dA, dB=dB, workspace=self.wsb), reps)
        return {"fwd_ms": round(f, 4), "bwd_ms": round(b, 4)}

    def extra(self, kernel_ms):
        out = {"cache_gather": gather_ceiling_report(self.gather_items, kernel_ms),
               "passes": self._pass_ms(self.B, self.C, self.dC, self.dA, self.dB)}
        if self.dtype == "f32":
            out["bf16"] = self._bf16_companion(kernel_ms)
        return out

    def _bf16_companion(self, f32_ms, steps=20):
        """The same step with B, C, dC and dB in BF16 (RNE of the FP32 draws; FP32 accumulation,
        dA in FP32) on the same handle, with the BF16 workload's pinned kernel shapes."""
        import torch
        from paper_2311_18141_amd import ops
        bf = torch.bfloat16
        self.Bb, self.dCb = self.B.to(bf), self.dC.to(bf)
        self.Cb = torch.empty(self.A.rows, self.N, dtype=bf, device=self.B.device)
        self.dBb = torch.empty_like(self.Bb)
        self.dAb = torch.empty_like(self.dA)
        pin = PINNED.get(self.name + "_bf16", {})
        cfg = {}
        if not AUTOTUNE and pin:
            kind, lanes, vec = pin["variant"]
            ops.spmm_tile_set_variant(self.tile, self.N, bf, kind, lanes, vec)
            kind, lanes, vec, depth = pin["bwd_variant"]
            ops.spmm_tile_set_bwd_variant(self.tile, self.N, bf, kind, lanes, vec, depth)
            cfg = {"variant": pin["variant"], "bwd_variant": pin["bwd_variant"], "pinned": True}
            fused = pin["bwd_variant"][0] == "fused"
        else:
            cfg["variant"] = ops.spmm_tile_autotune(self.tile, [self.Bb], self.Cb, tune_plan=False)
            cfg["bwd_variant"] = ops.spmm_tile_autotune_bwd(self.tile, self.dCb, self.dBb, B=self.Bb, dA=self.dAb)
            fused = cfg["bwd_variant"]["kind"] == "fused"
        self.wsf = self.tile.workspace(self.N, "fwd")
        self.wsb = self.tile.workspace(self.N, "bwd")

        def step():
            ops.spmm_fwd(self.tile, [self.Bb], C=self.Cb, workspace=self.wsf)
            ops.spmm_bwd(self.tile, self.dCb, self.Bb, dA=self.dAb, dB=self.dBb, workspace=self.wsb)

        for _ in range(3):
            step()
        ms = Batched._time(step, steps)
        traffic = stored_traffic(self.name, "bf16_hbm_bytes_per_step") if not AUTOTUNE else None
        return {"ms_per_step": round(ms, 5), "value": round(self.flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                "speedup_vs_f32": round(f32_ms / ms, 3), "kernels": cfg, "steps": steps,
                "traffic": traffic,
                "traffic_frac": round(traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "cache_gather": gather_ceiling_report(_fwdbwd_gather_items(self.A, self.N, 2, fused), ms),
                "passes": self._pass_ms(self.Bb, self.Cb, self.dCb, self.dAb, self.dBb),
                "note": "same handle and inputs as the FP32 step, B / C / dC / dB stored in BF16"}

    def accuracy(self):
        """Max and mean relative error of C, dA and dB against the FP64 oracle on a sample (2,000
        random rows of C with all their dA entries, 2,000 random rows of dB, plus the longest row
        and the most used column), after the timed region.  FP32 step: against the oracle on the
        FP32 operands.  BF16 companion: against the oracle on the FP32 operands (total error) and
        on the BF16-rounded operands (the kernels' own error)."""
        import torch
        import oracle
        A = self.A
        rng = np.random.Generator(np.random.PCG64(17))
        lens = A.row_lengths()
        cnt = np.bincount(A.colind, minlength=A.cols)
        rows = np.unique(np.concatenate([rng.choice(A.rows, 2000, replace=False), [int(np.argmax(lens))]]))
        cols = np.unique(np.concatenate([rng.choice(A.cols, 2000, replace=False), [int(np.argmax(cnt))]]))
        ents = np.concatenate([np.arange(A.rowptr[r], A.rowptr[r + 1], dtype=np.int64) for r in rows])
        dev = self.C.device
        r_t = torch.from_numpy(rows).to(dev)
        c_t = torch.from_numpy(cols).to(dev)
        e_t = torch.from_numpy(ents).to(dev)

        def one(C, dA, dB, Bh, dCh):
            rC, SC = oracle.spmm([(A.rowptr, A.colind, A.values)], [Bh], rows=rows)
            rA, SA = oracle.sddmm(A.rowptr, A.colind, dCh, Bh, entries=ents)
            rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dCh, out_rows=cols)
            return {name: _err_stats(got, ref, S)
                    for name, got, ref, S in (("C", C[r_t], rC, SC), ("dA", dA[e_t], rA, SA), ("dB", dB[c_t], rB, SB))}

        torch.cuda.synchronize()
        out = {"sample": "%d rows of C (%d dA entries), %d rows of dB" % (len(rows), len(ents), len(cols)),
               "definition": REL_DEFINITION}
        Bt = oracle.bf16_to_f32(oracle.f32_to_bf16(self.Bh))
        dCt = oracle.bf16_to_f32(oracle.f32_to_bf16(self.dCh))
        if self.dtype == "f32":
            out["f32"] = one(self.C, self.dA, self.dB, self.Bh, self.dCh)
            if hasattr(self, "Cb"):
                out["bf16_vs_f32_operands"] = one(self.Cb, self.dAb, self.dBb, self.Bh, self.dCh)
                out["bf16_vs_bf16_operands"] = one(self.Cb, self.dAb, self.dBb, Bt, dCt)
        else:
            out["bf16_vs_f32_operands"] = one(self.C, self.dA, self.dB, self.Bh, self.dCh)
            out["bf16_vs_bf16_operands"] = one(self.C, self.dA, self.dB, Bt, dCt)
        return out

    def cpu_sample(self):
        import oracle
        A, N = self.A, self.N
        lens = A.row_lengths()
        target = 0.6e10 / (2.0 * N)   # per pass; three passes
        r = int(min(A.rows, np.searchsorted(np.cumsum(lens), target) + 1))
        rows = np.arange(r, dtype=np.int64)
        nnz = int(lens[:r].sum())
        cols = np.arange(min(A.cols, r), dtype=np.int64)
        t0 = time.perf_counter()
        oracle.spmm([(A.rowptr, A.colind, A.values)], [self.Bh], rows=rows, scale=False)
        oracle.sddmm(A.rowptr, A.colind, self.dCh, self.Bh, entries=np.arange(nnz, dtype=np.int64))
        oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, self.dCh, out_rows=cols)
        dt = time.perf_counter() - t0
        nnz_t = float(np.isin(A.colind, cols).sum()) if A.nnz < 2e8 else float(nnz)
        flops = 2.0 * N * (2 * nnz + nnz_t)
        return flops, dt, ("oracle FP64 forward + SDDMM on rows [0, %d) and A^T dC on output rows [0, %d) of %d"
                           % (r, len(cols), A.rows))


class Batched(Workload):
    """Many independent uneven tiles in one batched launch: the single-launch form (one kernel for
    every item class, resident workgroups claiming items from per-XCD slices, split rows summed by
    a fix-up launch when a tile has them), per-tile variants from the autotuner; the per-tile launch loop (default and
    autotuned variants), the one-launch-per-class forms (flat and persistent hand-out) and the
    single launch with the flat hand-out are timed beside it, eagerly and as graph replays."""

    def __init__(self, name, count, config):
        self.name = name
        self.count = count
        self.config = config
        self.kernel = "spmm_batched (batch_union: one launch, persistent hand-out)"

    def setup(self):
        import torch
        import synth
        from paper_2311_18141_amd import ops
        t0 = time.time()
        self.tiles, self.Ns = synth.uneven_tiles(self.count, seed=self.config.get("seed", 4))
        _log("%s: %d tiles generated in %.1f s (nnz %d)" % (self.name, self.count, time.time() - t0,
                                                            sum(t.nnz for t in self.tiles)))
        rng = synth.streams(self.config.get("seed", 4))[3]
        dev = "cuda:0"
        self.handles, self.B, self.C, self.Bh = [], [], [], []
        for t, N in zip(self.tiles, self.Ns):
            b = synth.dense(t.cols, N, rng)
            self.Bh.append(b)
            self.B.append(torch.from_numpy(b).to(dev))
            self.C.append(torch.empty(t.rows, N, device=dev))
            d = (torch.from_numpy(t.rowptr).to(dev), torch.from_numpy(t.colind).to(dev),
                 torch.from_numpy(t.values).to(dev), t.cols)
            self.handles.append(ops.spmm_tile_create(t.rows, [d], validate=True, **_handle_opts(self.name)))
        torch.cuda.synchronize()
        # Reference point: one spmm_fwd launch per tile with the library's default variant.
        self.loop_ms = self._time(self._loop, reps=5)
        # The batch takes every tile's variant from the autotuner (part of its set-up; the
        # autotuner times the single-tile kernels, not the batch kernels timed below).
        t0 = time.time()
        for h, B, C in zip(self.handles, self.B, self.C):
            ops.spmm_tile_autotune(h, [B], C, tune_plan=False)
        _log("%s: autotuned %d tiles in %.1f s" % (self.name, self.count, time.time() - t0))
        self.batch = ops.spmm_batch_create(self.handles, self.Ns, single=True, persistent=True)
        self.ws = self.batch.workspace()
        # The other forms, timed for comparison, eagerly and as one captured HIP graph replayed:
        # one launch per item class with the flat (hardware dispatcher) or persistent (claim
        # counter) hand-out, and the single launch with the flat hand-out.
        self.forms_ms, self.graph_ms = {}, {"single_persistent": self._graph_ms(self.batch, self.ws)}
        for key, kw in (("per_class_flat", {}), ("per_class_persistent", {"persistent": True}),
                        ("single_flat", {"single": True})):
            ob = ops.spmm_batch_create(self.handles, self.Ns, **kw)
            ows = ob.workspace()
            self.forms_ms[key] = self._time(lambda: ops.spmm_batched(ob, self.B, self.C, workspace=ows), reps=5)
            self.graph_ms[key] = self._graph_ms(ob, ows)
            del ob, ows
        self.tuned_loop_ms = self._time(self._loop, reps=5)
        # each non-zero gathers its B row (4 N bytes) from the tile's B (cols x 4 N bytes)
        self.gather_items = [(float(t.nnz) * 4 * N, t.cols * 4 * N, 4 * N) for t, N in zip(self.tiles, self.Ns)]
        kinds = {}
        for t in range(self.count):
            v = self.batch.variant(t)
            key = "%s/%d/%d" % (v["kind"], v["lanes"], v["vec"])
            kinds[key] = kinds.get(key, 0) + 1
        nnz = sum(t.nnz for t in self.tiles)
        self.flops = sum(2.0 * t.nnz * N for t, N in zip(self.tiles, self.Ns))
        self.alg_bytes = float(sum(8 * t.nnz + 4 * (t.rows + 1) + 4 * (t.cols + t.rows) * N
                                   for t, N in zip(self.tiles, self.Ns)))
        self.config = dict(self.config, tiles=self.count, nnz=nnz, rows=sum(t.rows for t in self.tiles),
                           variants=kinds,
                           per_tile_loop={"ms": round(self.loop_ms, 4),
                                          "gflops": round(self.flops / (self.loop_ms * 1e-3) / 1e9, 1)},
                           per_tile_loop_autotuned={"ms": round(self.tuned_loop_ms, 4),
                                                    "gflops": round(self.flops / (self.tuned_loop_ms * 1e-3) / 1e9, 1)},
                           other_forms={k: {"ms": round(v, 4), "gflops": round(self.flops / (v * 1e-3) / 1e9, 1)}
                                        for k, v in self.forms_ms.items()},
                           graph_replay={k: {"ms": round(v, 4), "gflops": round(self.flops / (v * 1e-3) / 1e9, 1)}
                                         for k, v in self.graph_ms.items()})

    def _loop(self):
        from paper_2311_18141_amd import ops
        for h, B, C in zip(self.handles, self.B, self.C):
            ops.spmm_fwd(h, [B], C=C)

    def _graph_ms(self, batch, ws, reps=5):
        """Mean time of a replay of one captured spmm_batched call."""
        import torch
        from paper_2311_18141_amd import ops
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # operand arrays are built (and cached) outside the capture
            ops.spmm_batched(batch, self.B, self.C, workspace=ws)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ops.spmm_batched(batch, self.B, self.C, workspace=ws)
        ms = self._time(g.replay, reps)
        del g
        return ms

    def extra(self, kernel_ms):
        return {"cache_gather": gather_ceiling_report(self.gather_items, kernel_ms)}

    @staticmethod
    def _time(fn, reps):
        import torch
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def step(self):
        from paper_2311_18141_amd import ops
        ops.spmm_batched(self.batch, self.B, self.C, workspace=self.ws)

    def cpu_sample(self):
        import oracle
        flops, t_total, used = 0.0, 0.0, 0
        for t, N, b in zip(self.tiles, self.Ns, self.Bh):
            t0 = time.perf_counter()
            oracle.spmm([(t.rowptr, t.colind, t.values)], [b], scale=False)
            t_total += time.perf_counter() - t0
            flops += 2.0 * t.nnz * N
            used += 1
            if t_total > 15.0:
                break
        return flops, t_total, "oracle FP64 forward on the first %d of %d tiles" % (used, self.count)


# ---------------------------------------------------------------------------
# Gather ceiling: the rate at which whole rows of a dense table can be gathered at
# random (spmm_gather_probe: the forward's loads without its arithmetic), measured for
# table sizes that fit the L2s (4 MiB per XCD), the Infinity Cache (256 MiB) or only HBM.
# A workload's ceiling time is the sum over its parts of the bytes they gather at the
# probe rate for their row width and table size (interpolated in log2 of the size).
PROBE_MIB = (1, 4, 16, 64, 256, 1024, 4096)
_PROBE = {}


def _probe_rate(width, mib):
    import torch
    from paper_2311_18141_amd import ops
    key = (width, mib)
    if key not in _PROBE:
        dev = "cuda:0"
        gen = torch.Generator(device=dev)
        gen.manual_seed(11)
        size = mib << 20
        table = torch.randint(-(1 << 31), (1 << 31) - 1, (size // 4,), dtype=torch.int32, device=dev, generator=gen)
        n = min(1 << 24, (2 << 30) // width)
        idx = torch.randint(0, size // width, (n,), dtype=torch.int32, device=dev, generator=gen)
        out = torch.empty(1, dtype=torch.int32, device=dev)
        ms = Batched._time(lambda: ops.spmm_gather_probe(table, width, idx, out), reps=3)
        _PROBE[key] = n * width / (ms * 1e-3)
        del table, idx
    return _PROBE[key]


def _probe_width(row_bytes):
    """The probe row for a gather of row_bytes: capped at 1 KiB (the widest rows here)."""
    w = min(int(row_bytes), 1024)
    return max(16, w - w % 16)


def gather_ceiling_report(items, kernel_ms):
    """items: (bytes gathered, table bytes, row bytes) per part of a step."""
    lg = np.log2(np.array(PROBE_MIB, dtype=np.float64))
    total, ceil_s, used = 0.0, 0.0, {}
    for g, table, row in items:
        w = _probe_width(row)
        x = float(np.clip(np.log2(max(table, 1) / float(1 << 20)), lg[0], lg[-1]))
        k = int(np.searchsorted(lg, x))
        lo, hi = max(k - 1, 0), min(k, len(lg) - 1)
        if lg[hi] == x:
            lo = hi
        r_lo, r_hi = _probe_rate(w, PROBE_MIB[lo]), _probe_rate(w, PROBE_MIB[hi])
        rate = r_lo if hi == lo else r_lo + (r_hi - r_lo) * (x - lg[lo]) / (lg[hi] - lg[lo])
        for m in (PROBE_MIB[lo], PROBE_MIB[hi]):
            used.setdefault("%dB" % w, {})["%dMiB" % m] = round(_PROBE[(w, m)] / 1e9, 1)
        total += g
        ceil_s += g / rate
    return {"probe": "spmm_gather_probe: random whole rows (up to 1 KiB) of a table of the part's size",
            "probe_GBps": used,
            "gathered_GB": round(total / 1e9, 2),
            "achieved_GBps": round(total / (kernel_ms * 1e-3) / 1e9, 1),
            "ceiling_ms": round(ceil_s * 1e3, 3),
            "frac": round(ceil_s * 1e3 / kernel_ms, 4)}



class StationaryA(Workload):
    """The stationary-A local step (Section 3.2, Algorithm 1) on one GPU: the owner of A(i,k)
    forms the partial products P_j = A(i,k) B(k,j) (accumulate = 0) for every column block j,
    and the owner of each C(i,j) adds its partial (spmm_tile_accumulate).  Here both owners are
    this GPU: tile (0,0) of the R-MAT scale-22 4 x 4 grid against 4 column blocks of N = 128."""

    def __init__(self, name, config):
        self.name = name
        self.config = config
        self.kernel = "spmm_fwd (partials) + spmm_tile_accumulate"

    def setup(self):
        import torch
        import synth
        from paper_2311_18141_amd import ops
        t0 = time.time()
        self.A = synth.rmat_row_block(22, 16, 4, 0, seed=2).tiles[0]
        A = self.A
        _log("%s: inputs generated in %.1f s (nnz %d)" % (self.name, time.time() - t0, A.nnz))
        self.N, self.J = 128, 4
        rng = synth.streams(2)[2]
        dev = "cuda:0"
        self.Bh = [synth.dense(A.cols, self.N, rng) for _ in range(self.J)]
        self.B = [torch.from_numpy(b).to(dev) for b in self.Bh]
        self.C = [torch.from_numpy(synth.dense(A.rows, self.N, rng)).to(dev) for _ in range(self.J)]
        self.P = [torch.empty(A.rows, self.N, device=dev) for _ in range(self.J)]
        d = (torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev),
             torch.from_numpy(A.values).to(dev), A.cols)
        self.tile = ops.spmm_tile_create(A.rows, [d], validate=True, **_handle_opts("rmat22_rowblock0_4x4_n128"))
        self.config["variant"] = _apply_pin("rmat22_rowblock0_4x4_n128", self.tile, self.N, torch.float32)
        self.ws = self.tile.workspace(self.N)
        self.flops = 2.0 * A.nnz * self.N * self.J
        fwd = 8 * A.nnz + 4 * (A.rows + 1) + 4 * (A.cols + A.rows) * self.N
        acc = 3 * 4 * A.rows * self.N
        self.alg_bytes = float(self.J * (fwd + acc))
        self.config = dict(self.config, nnz=A.nnz, rows=A.rows, N=self.N, column_blocks=self.J)

    def step(self):
        from paper_2311_18141_amd import ops
        for j in range(self.J):
            ops.spmm_fwd(self.tile, [self.B[j]], C=self.P[j], workspace=self.ws)
            ops.spmm_tile_accumulate(self.C[j], self.P[j])

    def cpu_sample(self):
        import oracle
        A = self.A
        lens = A.row_lengths()
        target = 2.0e10 / (2.0 * self.N)
        r = int(min(A.rows, np.searchsorted(np.cumsum(lens), target) + 1))
        rows = np.arange(r, dtype=np.int64)
        t0 = time.perf_counter()
        oracle.spmm([(A.rowptr, A.colind, A.values)], [self.Bh[0]], rows=rows, scale=False)
        dt = time.perf_counter() - t0
        return 2.0 * float(lens[:r].sum()) * self.N, dt, "oracle FP64 partial product on rows [0, %d)" % r


class StationaryAGrid(Workload):
    """The stationary-A step of one row block with work stealing (Section 3.4, Algorithm 3), on one
    GPU: row block 0 of the R-MAT scale-22 4 x 4 grid, A(0,k) for k = 0..3 (the stationary
    tiles, nnz 20.7M / 7.1M / 7.1M / 2.4M), against B(k,j) for 4 column blocks j of N = 128.
    The 16 component products A(0,k) B(k,j) form one batch handed out through a 3-D
    reservation grid over (0, j, k) (locality-aware stealing): workers (waves of resident
    workgroups, owners by XCD) take the items of their own products with one fetch-and-add per
    item, then those sharing their C tile, A tile, B tile, then the rest; each product writes a
    partial tile, and the owner of C(0,j) drains its four partials in k order
    (spmm_tile_accumulate_n).  Beside it: the 2-D grid over (0, k) (random stealing), the 2-D
    grid without stealing, the single launch without a grid, and one spmm_fwd launch per
    product (the static order)."""

    def __init__(self, name, config):
        self.name = name
        self.config = config
        self.kernel = "spmm_batched (batch_reserve, 3-D grid) + spmm_tile_accumulate_n"

    def setup(self):
        import torch
        import synth
        from paper_2311_18141_amd import ops
        t0 = time.time()
        self.As = synth.rmat_row_block(22, 16, 4, 0, seed=2).tiles
        K, J, N = len(self.As), 4, 128
        self.K, self.J, self.N = K, J, N
        rows = self.As[0].rows
        _log("%s: inputs generated in %.1f s (nnz %d)" % (self.name, time.time() - t0, sum(a.nnz for a in self.As)))
        dev = "cuda:0"
        rng = synth.streams(2)[2]
        self.handles = []
        for A in self.As:
            d = (torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev),
                 torch.from_numpy(A.values).to(dev), A.cols)
            h = ops.spmm_tile_create(rows, [d], validate=True, **_handle_opts("rmat22_rowblock0_4x4_n128"))
            _apply_pin("rmat22_rowblock0_4x4_n128", h, N, torch.float32)
            self.handles.append(h)
        self.Bh = [[synth.dense(A.cols, N, rng) for _ in range(J)] for A in self.As]
        self.C0 = [synth.dense(rows, N, rng) for _ in range(J)]
        self.Bd, self.Pd, tiles, coords = [], [], [], []
        for k in range(K):
            for j in range(J):
                self.Bd.append(torch.from_numpy(self.Bh[k][j]).to(dev))
                self.Pd.append(torch.empty(rows, N, device=dev))
                tiles.append(self.handles[k])
                coords.append((0, j, k))
        self.C = [torch.from_numpy(c).to(dev) for c in self.C0]
        self.batches = {m: ops.spmm_batch_create_grid(tiles, [N] * len(tiles), coords, m) for m in ("2d", "3d", "own")}
        self.batches["single"] = ops.spmm_batch_create(tiles, [N] * len(tiles), single=True, persistent=True)
        self.ws = {m: b.workspace() for m, b in self.batches.items()}
        self.fws = [h.workspace(N) for h in self.handles]
        nnz = sum(a.nnz for a in self.As)
        self.flops = 2.0 * nnz * N * J
        prod = sum(J * (8 * a.nnz + 4 * (rows + 1)) + 4 * a.cols * N * J + 4 * rows * N * J for a in self.As)
        acc = J * (2 + K) * 4 * rows * N
        self.alg_bytes = float(prod + acc)
        torch.cuda.synchronize()
        self.forms_ms = {}
        for m in ("2d", "own", "single", "loop"):
            self.forms_ms[m] = Batched._time(lambda: self._run(m), reps=3)
        self.config = dict(self.config, nnz=nnz, rows=rows, N=N, k_tiles=K, column_blocks=J,
                           nnz_per_k=[a.nnz for a in self.As],
                           other_forms={m: {"ms": round(v, 4), "gflops": round(self.flops / (v * 1e-3) / 1e9, 1)}
                                        for m, v in self.forms_ms.items()},
                           forms="the step: 3-D reservation grid (locality-aware stealing); 2d: 2-D grid "
                                 "(random stealing); own: 2-D grid, no stealing; single: one launch, per-XCD "
                                 "slices, no grid; loop: one spmm_fwd per product (the static order)")

    def _run(self, mode):
        from paper_2311_18141_amd import ops
        if mode == "loop":
            for t in range(self.K * self.J):
                ops.spmm_fwd(self.handles[t // self.J], [self.Bd[t]], C=self.Pd[t], workspace=self.fws[t // self.J])
        else:
            ops.spmm_batched(self.batches[mode], self.Bd, self.Pd, workspace=self.ws[mode])
        for j in range(self.J):
            ops.spmm_tile_accumulate_n(self.C[j], [self.Pd[k * self.J + j] for k in range(self.K)])

    def step(self):
        self._run("3d")

    def cpu_sample(self):
        import oracle
        lens = sum(a.row_lengths() for a in self.As)
        target = 2.0e10 / (2.0 * self.N)
        r = int(min(self.As[0].rows, np.searchsorted(np.cumsum(lens), target) + 1))
        rows = np.arange(r, dtype=np.int64)
        t0 = time.perf_counter()
        oracle.spmm([(a.rowptr, a.colind, a.values) for a in self.As], [self.Bh[k][0] for k in range(self.K)],
                    rows=rows, scale=False)
        dt = time.perf_counter() - t0
        return 2.0 * float(lens[:r].sum()) * self.N, dt, "oracle FP64 C(0,0) rows [0, %d) over the 4 k-tiles" % r


class SpgemmAA(Workload):
    """Local SpGEMM C = A A (the local step of the paper's SpGEMM experiments).  A step is the
    numeric phase (spgemm_compute); the symbolic phase (plan creation) is timed beside it."""

    metric = "SpGEMM GFLOP/s (2 * products) and % HBM roofline"

    def __init__(self, name, make, config):
        self.name = name
        self.make = make
        self.config = config
        self.kernel = "spgemm_compute (num_wave / num_block / num_window)"

    def setup(self):
        import torch
        from paper_2311_18141_amd import ops
        t0 = time.time()
        self.A = self.make()
        A = self.A
        _log("%s: inputs generated in %.1f s (nnz %d)" % (self.name, time.time() - t0, A.nnz))
        dev = "cuda:0"
        self.d = (torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev),
                  torch.from_numpy(A.values).to(dev), A.cols)
        torch.cuda.synchronize()
        ops.spgemm_create(A.rows, self.d, self.d, validate=True)  # first call: code objects, allocator
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            t0 = time.perf_counter()
            plan = ops.spgemm_create(A.rows, self.d, self.d, validate=False)
            torch.cuda.synchronize()
            reps.append((time.perf_counter() - t0) * 1e3)
            if _ < 2:
                del plan
        self.plan = plan
        self.symbolic_ms = min(reps)
        self.ci = torch.empty(max(plan.nnz_c, 1), dtype=torch.int32, device=dev)
        self.va = torch.empty(max(plan.nnz_c, 1), dtype=torch.float32, device=dev)
        self.flops = 2.0 * plan.products
        M = A.rows
        self.alg_bytes = float(2 * (8 * A.nnz + 4 * (M + 1)) + 8 * plan.nnz_c + 4 * (M + 1))
        self.config = dict(self.config, rows=M, nnz=A.nnz, products=plan.products, nnz_c=plan.nnz_c,
                           compression=round(plan.products / max(plan.nnz_c, 1), 3),
                           symbolic_ms=round(self.symbolic_ms, 3))

    def step(self):
        from paper_2311_18141_amd import ops
        ops.spgemm_compute(self.plan, self.ci, self.va)

    def extra(self, kernel_ms):
        """The local SpGEMM roofline of Section 4 (Gu et al.): arithmetic intensity
        cf / ((3 + 2 cf) b) with cf the multiply-adds per output entry and b = 8 bytes per
        entry (int32 index, FP32 value), i.e. (3 + 2 cf) b bytes per output entry, each
        product reading its B entry; its time at the HBM peak against the measured one."""
        nnz_c = max(self.plan.nnz_c, 1)
        cf = self.plan.products / nnz_c
        b = 8.0
        bytes_step = nnz_c * (3.0 + 2.0 * cf) * b
        t_ms = bytes_step / (HBM_PEAK_GBS * 1e9) * 1e3
        return {"local_spgemm_roofline": {"cf": round(cf, 3), "ai_products_per_byte": round(cf / ((3 + 2 * cf) * b), 5),
                                          "bytes_per_step": bytes_step, "time_at_peak_ms": round(t_ms, 3),
                                          "frac": round(t_ms / kernel_ms, 4)},
                "plan_reuse": self._plan_reuse(kernel_ms)}

    def _plan_reuse(self, kernel_ms):
        """Plan creation and compute calls with C's column pattern kept (the step above: every
        call after the first) and without (keep_pattern=False: columns found on every call).
        A plan's first call finds the columns either way and, when kept, copies them into the
        plan, so keeping them costs that copy once."""
        import torch
        from paper_2311_18141_amd import ops
        A = self.A

        def first_call(keep):
            t0 = time.perf_counter()
            plan = ops.spgemm_create(A.rows, self.d, self.d, validate=False, keep_pattern=keep)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ops.spgemm_compute(plan, self.ci, self.va)
            e1.record()
            torch.cuda.synchronize()
            return plan, (t1 - t0) * 1e3, e0.elapsed_time(e1)

        best = {}
        for keep in (True, False):
            for _ in range(2):
                plan, c_ms, f_ms = first_call(keep)
                if keep not in best or c_ms + f_ms < sum(best[keep][1:]):
                    best[keep] = (plan.pattern_entries, c_ms, f_ms)
                if not keep:
                    later = Batched._time(lambda: ops.spgemm_compute(plan, self.ci, self.va), 5)
                del plan
        out = {}
        for keep, name, calls in ((True, "kept_pattern", kernel_ms), (False, "bitmap_only", later)):
            ent, c_ms, f_ms = best[keep]
            out[name] = {"create_ms": round(c_ms, 3), "first_call_ms": round(f_ms, 4), "later_call_ms": round(calls, 4),
                         "create_and_one_call_ms": round(c_ms + f_ms, 3), "entries_kept": ent}
        return out

    def cpu_sample(self):
        import oracle
        A = self.A
        L = A.row_lengths()
        fl = np.bincount(np.repeat(np.arange(A.rows), L), weights=L[A.colind], minlength=A.rows)
        r = int(min(A.rows, np.searchsorted(np.cumsum(fl), 1.0e10) + 1))  # the whole matrix here (a few s)
        rows = np.arange(r, dtype=np.int64)
        t0 = time.perf_counter()
        oracle.spgemm((A.rowptr, A.colind, A.values), (A.rowptr, A.colind, A.values), A.cols, rows=rows, scale=False)
        dt = time.perf_counter() - t0
        return 2.0 * float(fl[:r].sum()), dt, "oracle FP64 SpGEMM on rows [0, %d) of %d" % (r, A.rows)


class CopyCalibration(Workload):
    """A plain device copy of 1 GiB: the reference against which HBM counters are scaled."""

    def __init__(self):
        self.name = "copy_1gib"
        self.kernel = "device copy (torch copy_)"
        self.config = {"workload": "copy_1gib", "bytes_read": 1 << 30, "bytes_written": 1 << 30}

    def setup(self):
        import torch
        self.x = torch.ones(1 << 28, device="cuda:0")
        self.y = torch.empty_like(self.x)
        self.flops = 0.0
        self.alg_bytes = float(2 << 30)

    def step(self):
        self.y.copy_(self.x)

    def cpu_sample(self):
        x = np.ones(1 << 26, dtype=np.float32)
        t0 = time.perf_counter()
        y = x.copy()
        dt = time.perf_counter() - t0
        return 0.0, dt, "numpy copy of 256 MiB (%.0f)" % float(y[0])


class GatherCalibration(Workload):
    """spmm_gather_probe over a table of known size: n random whole rows, every byte of each
    row read once (plus the 4-byte index), so the bytes a counter should see are known.  Used to
    calibrate the HBM counters for gathers of the row widths the kernels issue."""

    def __init__(self, row_bytes, table_mib, n):
        self.row_bytes, self.table_mib, self.n = row_bytes, table_mib, n
        self.name = "gather_%db_%dmib" % (row_bytes, table_mib)
        self.kernel = "spmm_gather_probe (probe_gather_kernel)"
        self.config = {"workload": self.name, "row_bytes": row_bytes, "table_bytes": table_mib << 20, "rows_gathered": n}

    def setup(self):
        import torch
        dev = "cuda:0"
        gen = torch.Generator(device=dev)
        gen.manual_seed(11)
        size = self.table_mib << 20
        self.table = torch.randint(-(1 << 31), (1 << 31) - 1, (size // 4,), dtype=torch.int32, device=dev,
                                   generator=gen)
        self.idx = torch.randint(0, size // self.row_bytes, (self.n,), dtype=torch.int32, device=dev, generator=gen)
        self.out = torch.empty(1, dtype=torch.int32, device=dev)
        self.flops = 0.0
        self.alg_bytes = float(self.n) * (self.row_bytes + 4)
        self.metric = "gathered GB/s"

    def step(self):
        from paper_2311_18141_amd import ops
        ops.spmm_gather_probe(self.table, self.row_bytes, self.idx, self.out)

    def cpu_sample(self):
        t = self.table[: 1 << 20].cpu().numpy()
        i = self.idx[: 1 << 20].cpu().numpy() % (t.size * 4 // self.row_bytes)
        t0 = time.perf_counter()
        x = np.bitwise_xor.reduce(t.view(np.uint8).reshape(-1, self.row_bytes)[i].view(np.uint32).ravel())
        dt = time.perf_counter() - t0
        return 0.0, dt, "numpy gather of 2^20 rows (xor %d)" % int(x)


def workloads():
    import synth
    return {
        "copy_1gib": lambda: CopyCalibration(),
        "gather_512b_4096mib": lambda: GatherCalibration(512, 4096, 1 << 23),
        "gather_128b_4096mib": lambda: GatherCalibration(128, 4096, 1 << 25),
        "gather_16b_4096mib": lambda: GatherCalibration(16, 4096, 1 << 26),
        "stationary_a_rmat22_rowblock0_4x4_grid": lambda: StationaryAGrid(
            "stationary_a_rmat22_rowblock0_4x4_grid",
            {"workload": "stationary_a_rmat22_rowblock0_4x4_grid", "matrix": "row block 0 of the R-MAT scale 22, "
             "edge factor 16 4x4 grid (4 stationary tiles A(0,k)) against 4 column blocks of N = 128", "seed": 2}),
        "stationary_a_rmat22_tile00_n128x4": lambda: StationaryA(
            "stationary_a_rmat22_tile00_n128x4",
            {"workload": "stationary_a_rmat22_tile00_n128x4", "matrix": "tile (0,0) of the R-MAT scale 22, "
             "edge factor 16 4x4 grid; 4 column blocks of N = 128", "seed": 2}),
        "spgemm_rmat18_ef16_aa": lambda: SpgemmAA(
            "spgemm_rmat18_ef16_aa", lambda: synth.rmat_csr(18, 16, seed=7),
            {"workload": "spgemm_rmat18_ef16_aa", "matrix": "R-MAT scale 18, edge factor 16, "
             "(0.57,0.19,0.19,0.05), C = A A", "seed": 7}),
        "spgemm_er1m16_aa": lambda: SpgemmAA(
            "spgemm_er1m16_aa", lambda: synth.uniform_csr(1 << 20, 1 << 20, 16, seed=8),
            {"workload": "spgemm_er1m16_aa", "matrix": "1,048,576^2 uniform, 16 nnz/row, C = A A", "seed": 8}),
        "uneven512_batched": lambda: Batched(
            "uneven512_batched", 512,
            {"workload": "uneven512_batched", "matrix": "512 square tiles, rows log-uniform in [1024, 65536], "
             "r_t uniform in [4, 256] non-zeros per row, N_t in {32, 64, 128, 256}", "seed": 4}),
        "rmat22_rowblock0_4x4_n128": lambda: TileRowForward(
            "rmat22_rowblock0_4x4_n128",
            lambda: synth.rmat_row_block(22, 16, 4, 0, seed=2).tiles, 128, "f32",
            {"workload": "rmat22_rowblock0_4x4_n128", "matrix": "R-MAT scale 22, edge factor 16, "
             "(0.57,0.19,0.19,0.05), row block 0 of a 4x4 tile grid", "seed": 2, "column_panels": [2, 4, 8]}),
        "er4096_n32": lambda: TileRowForward(
            "er4096_n32", lambda: [synth.uniform_csr(4096, 4096, 16, seed=1)], 32, "f32",
            {"workload": "er4096_n32", "matrix": "4096^2 uniform, 16 nnz/row", "seed": 1}),
        "rmat23_n256_bf16": lambda: TileRowForward(
            "rmat23_n256_bf16", lambda: [synth.rmat_csr(23, 32, seed=5)], 256, "bf16",
            {"workload": "rmat23_n256_bf16", "matrix": "R-MAT scale 23, edge factor 32", "seed": 5}),
        "rmat23_n256_f32": lambda: TileRowForward(
            "rmat23_n256_f32", lambda: [synth.rmat_csr(23, 32, seed=5)], 256, "f32",
            {"workload": "rmat23_n256_f32", "matrix": "R-MAT scale 23, edge factor 32", "seed": 5}),
        "powerlaw2m_n128_fwdbwd_bf16": lambda: ForwardBackward(
            "powerlaw2m_n128_fwdbwd_bf16", lambda: synth.powerlaw_csr(1 << 21, 1 << 21, 32, 65536, seed=3), 128,
            {"workload": "powerlaw2m_n128_fwdbwd_bf16", "matrix": "2,097,152^2, Pareto(2.1) row degrees, mean 32, "
             "max 65,536, values N(0,1)/sqrt(deg); B, C, dC, dB in BF16", "seed": 3}, dtype="bf16"),
        "powerlaw2m_n128_fwdbwd": lambda: ForwardBackward(
            "powerlaw2m_n128_fwdbwd", lambda: synth.powerlaw_csr(1 << 21, 1 << 21, 32, 65536, seed=3), 128,
            {"workload": "powerlaw2m_n128_fwdbwd", "matrix": "2,097,152^2, Pareto(2.1) row degrees, mean 32, "
             "max 65,536, values N(0,1)/sqrt(deg)", "seed": 3}),
        "powerlaw2m_n512_fwdbwd": lambda: ForwardBackward(
            "powerlaw2m_n512_fwdbwd", lambda: synth.powerlaw_csr(1 << 21, 1 << 21, 32, 65536, seed=3), 512,
            {"workload": "powerlaw2m_n512_fwdbwd", "matrix": "2,097,152^2, Pareto(2.1) row degrees, mean 32, "
             "max 65,536, values N(0,1)/sqrt(deg); N = 512: the library's default shapes, the fused backward "
             "in two 256-column windows", "seed": 3}),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="powerlaw2m_n128_fwdbwd")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--long-row", type=int, default=0, help="split-row threshold (0 = library default)")
    ap.add_argument("--segment", type=int, default=0, help="non-zeros per split unit (0 = library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="re-tune variant and split plan in set-up instead of the pinned ones")
    args = ap.parse_args()
    global AUTOTUNE
    AUTOTUNE = args.autotune
    HANDLE_OPTS.update(long_row=args.long_row, segment=args.segment)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the stationary-C tile row is "
              "one GPU's share); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    wl = workloads()[args.workload]()
    wl.setup()
    torch.cuda.synchronize()
    _log("setup done; warmup %d" % args.warmup)
    for _ in range(args.warmup):
        wl.step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_all0.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        wl.step()
        ev[i][1].record(stream)
    t_all1.record(stream)
    torch.cuda.synchronize()
    ms_total = t_all0.elapsed_time(t_all1)
    per = [a.elapsed_time(b) for a, b in ev]
    ms_step = ms_total / args.steps
    value = wl.flops / (ms_step * 1e-3) / 1e9 if wl.flops else wl.alg_bytes / (ms_step * 1e-3) / 1e9
    avg_kernel_ms = float(np.mean(per))
    achieved = wl.alg_bytes / (avg_kernel_ms * 1e-3) / 1e9
    _log("timed %d steps: %.4f ms/step (per-step events mean %.4f, min %.4f, max %.4f)"
         % (args.steps, ms_step, avg_kernel_ms, min(per), max(per)))
    traffic = stored_traffic(args.workload)
    out = {
        "metric": wl.metric,
        "value": round(value, 2),
        "unit": "GFLOP/s" if wl.flops else "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl.dtype,
        "data": "synthetic",
        "config": wl.config,
        "roofline": {"bound": "hbm", "kernel": wl.kernel, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_step": wl.alg_bytes,
                     "avg_kernel_ms": round(avg_kernel_ms, 5),
                     # counter-measured HBM bytes per step over the same time, against the same peak
                     "traffic_frac": (round(traffic / (avg_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None)},
    }
    out.update(wl.extra(avg_kernel_ms))
    if not args.no_cpu_baseline:
        # The oracle legs: its time on the host cores, and (for workloads that define it) the
        # error of the step's results against it on a sample, both after the timed region.
        threads = _threads()
        os.environ["OMP_NUM_THREADS"] = str(threads)
        flops, secs, desc = wl.cpu_sample()
        out["cpu_baseline"] = {"value": round(flops / secs / 1e9, 3), "unit": "GFLOP/s", "cores": threads,
                               "kind": "oracle", "sample": desc, "seconds": round(secs, 2),
                               "cpu_model": _cpu_model()}
        if hasattr(wl, "accuracy"):
            t0 = time.time()
            out["accuracy"] = wl.accuracy()
            _log("accuracy sample in %.1f s" % (time.time() - t0))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
