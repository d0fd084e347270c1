"""Guard bands around every output, input and workspace.  Each operand lives inside a larger
block whose other elements (a band before and after it, and the padding columns of a leading
dimension wider than the row) hold a NaN canary; after the call every canary of an output is
intact, every input block (canaries and data) is unchanged, and the interior matches the FP64
oracle.  Covers the forward (several k-tiles, split long rows, hot-row staging, each kernel
family, BF16), the backward (dA and dB), the batched launch in both hand-out modes, the
owner-side accumulate and the local SpGEMM.  A band of one element leaves an operand only
element-aligned, which drives the narrow-vector variants."""
import numpy as np
import pytest
import torch

import oracle
import synth

from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu

# canary bit patterns: a quiet NaN of each float type (never a result of the arithmetic on
# finite inputs), an out-of-range index for int32
_CANARY = {torch.float32: (torch.int32, 0x7FBADBAD), torch.bfloat16: (torch.int16, 0x7FBD),
           torch.int32: (torch.int32, -0x21524111), torch.uint8: (torch.uint8, 0xA5)}


class Guarded:
    """A rows x N matrix (leading dimension ld) inside one flat block with `band` canary
    elements on each side; its padding columns hold canaries too."""

    def __init__(self, rows, N, dtype, ld=None, band=64):
        ld = N if ld is None else ld
        raw_dt, self.pat = _CANARY[dtype]
        n = band + rows * ld + band
        self.raw = torch.full((n,), self.pat, dtype=raw_dt, device=G.DEV)
        flat = self.raw.view(dtype) if raw_dt != dtype else self.raw
        self.view = flat[band: band + rows * ld].view(rows, ld)[:, :N] if rows * ld else flat[band:band].view(rows, N)
        mask = torch.ones(n, dtype=torch.bool)
        if rows * ld:
            mask[band: band + rows * ld].view(rows, ld)[:, :N] = False
        self.mask = mask.to(G.DEV)

    def set(self, host):
        self.view.copy_(torch.from_numpy(np.ascontiguousarray(host)).to(self.view.dtype))
        self.before = self.raw.clone()
        return self

    def canaries_intact(self):
        return bool((self.raw[self.mask] == self.pat).all())

    def unchanged(self):
        return torch.equal(self.raw, self.before)


def _ws(nbytes):
    """A workspace slice of exactly nbytes with 256-byte canary bands (None when 0)."""
    if nbytes == 0:
        return None, None
    g = Guarded(1, nbytes, torch.uint8, band=256)
    return g, g.view[0]


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _tile_row(seed, rows=700, cols=(300, 1200, 2000), long_rows=True):
    rng = _rng(seed)
    As = []
    for c in cols:
        L = rng.integers(0, 40, size=rows)
        if long_rows:
            L[rng.choice(rows, size=4, replace=False)] = min(c, 1000)
        L[rng.choice(rows, size=20, replace=False)] = 0
        As.append(synth.random_csr(rows, c, L, rng, "int8"))
    return As


def _check_fwd_interior(got, ref, S, dtype, As):
    if dtype == torch.float32:
        assert np.array_equal(got.astype(np.float64), ref)
    else:
        G.assert_bf16_close(got, ref, S)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("band", [64, 1])
@pytest.mark.parametrize("variant", [None, ("stream", 0, 1), ("stream", 0, 4), ("rowsplit", 8, 0),
                                     ("rowsplit", 64, 0)])
@pytest.mark.parametrize("N", [7, 64])
def test_fwd_guard_bands(dtype, band, variant, N):
    G.note("canary fwd dtype=%s band=%d variant=%s N=%d" % (dtype, band, variant, N))
    As = _tile_row(1)
    tile = G.make_tile(As, long_row=256, segment=100, hot_rows=32)
    assert tile.stats()["hot_rows"] > 0
    if variant is not None:
        ops.spmm_tile_set_variant(tile, N, dtype, *variant)
    rng = _rng(2)
    Bh = [synth.dense(A.cols, N, rng, "int8") for A in As]
    C0 = synth.dense(As[0].rows, N, rng, "int8")
    Bg = [Guarded(A.cols, N, dtype, ld=N + 5, band=band).set(b) for A, b in zip(As, Bh)]
    for accumulate in (False, True):
        Cg = Guarded(As[0].rows, N, dtype, ld=N + 3, band=band).set(C0)
        wsg, ws = _ws(ops.spmm_fwd_workspace_bytes(tile, N))
        ops.spmm_fwd(tile, [g.view for g in Bg], C=Cg.view, k_offset=1, accumulate=accumulate, workspace=ws)
        torch.cuda.synchronize()
        assert Cg.canaries_intact(), accumulate
        assert wsg is None or wsg.canaries_intact()
        assert all(g.unchanged() for g in Bg)
        Bref = Bh if dtype == torch.float32 else [G.bf16_as_f32(b) for b in Bh]
        ref, S = G.oracle_fwd(As, Bref, k_offset=1, accumulate=accumulate, C0=C0)
        _check_fwd_interior(G.host_f32(Cg.view), ref, S, dtype, As)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("band", [64, 1])
@pytest.mark.parametrize("N", [5, 128])
def test_bwd_guard_bands(dtype, band, N):
    G.note("canary bwd dtype=%s band=%d N=%d" % (dtype, band, N))
    A = _tile_row(3, rows=900, cols=(1500,))[0]
    tile = G.make_tile([A], transpose=True, long_row=256, segment=100)
    rng = _rng(4)
    dCh = synth.dense(A.rows, N, rng, "int8")
    Bh = synth.dense(A.cols, N, rng, "int8")
    dCg = Guarded(A.rows, N, dtype, ld=N + 9, band=band).set(dCh)
    Bg = Guarded(A.cols, N, dtype, ld=N + 1, band=band).set(Bh)
    dAg = Guarded(1, A.nnz, torch.float32, band=band)
    dBg = Guarded(A.cols, N, dtype, ld=N + 3, band=band)
    wsg, ws = _ws(ops.spmm_bwd_workspace_bytes(tile, N))
    ops.spmm_bwd(tile, dCg.view, Bg.view, dA=dAg.view[0], dB=dBg.view, workspace=ws)
    torch.cuda.synchronize()
    assert dAg.canaries_intact() and dBg.canaries_intact()
    assert wsg is None or wsg.canaries_intact()
    assert dCg.unchanged() and Bg.unchanged()
    # int8 data: every product and partial sum is an integer far below 2^24, exact in FP32
    dA_ref, _ = oracle.sddmm(A.rowptr, A.colind, dCh, Bh)
    assert np.array_equal(G.host_f32(dAg.view[0]).astype(np.float64), dA_ref)
    dB_ref, S = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dCh)
    got = G.host_f32(dBg.view)
    if dtype == torch.float32:
        assert np.array_equal(got.astype(np.float64), dB_ref)
    else:
        G.assert_bf16_close(got, dB_ref, S)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("persistent,single", [(False, False), (True, False), (False, True), (True, True)])
def test_batched_guard_bands(dtype, persistent, single):
    G.note("canary batched dtype=%s persistent=%s single=%s" % (dtype, persistent, single))
    rng = _rng(5)
    As, Ns = [], [32, 64, 128, 256, 64, 32, 128, 8]
    for t, N in enumerate(Ns):
        rows = int(rng.integers(50, 3000))
        L = rng.integers(0, 50, size=rows)
        L[rng.integers(0, rows, size=2)] = min(rows, 900)
        As.append(synth.random_csr(rows, rows, L, rng, "int8"))
    handles = [G.make_tile([A], long_row=256, segment=128) for A in As]
    batch = ops.spmm_batch_create(handles, Ns, dtype, persistent=persistent, single=single)
    Bh = [synth.dense(A.cols, N, rng, "int8") for A, N in zip(As, Ns)]
    C0 = [synth.dense(A.rows, N, rng, "int8") for A, N in zip(As, Ns)]
    # rows start on 16-byte boundaries, as the batched launch requires
    Bg = [Guarded(A.cols, N, dtype, ld=N + 8, band=64).set(b) for A, N, b in zip(As, Ns, Bh)]
    Cg = [Guarded(A.rows, N, dtype, ld=N + 16, band=64).set(c) for A, N, c in zip(As, Ns, C0)]
    wsg, ws = _ws(batch.workspace_bytes())
    ops.spmm_batched(batch, [g.view for g in Bg], [g.view for g in Cg], accumulate=True, workspace=ws)
    torch.cuda.synchronize()
    assert all(g.canaries_intact() for g in Cg)
    assert wsg is None or wsg.canaries_intact()
    assert all(g.unchanged() for g in Bg)
    for t, A in enumerate(As):
        Bref = Bh[t] if dtype == torch.float32 else G.bf16_as_f32(Bh[t])
        ref, S = G.oracle_fwd([A], [Bref], accumulate=True, C0=C0[t])
        _check_fwd_interior(G.host_f32(Cg[t].view), ref, S, dtype, [A])


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("band", [64, 1])
def test_accumulate_guard_bands(dtype, band):
    G.note("canary accumulate dtype=%s band=%d" % (dtype, band))
    rng = _rng(6)
    rows, N = 1000, 24
    Ch = synth.dense(rows, N, rng, "int8")
    Ph = synth.dense(rows, N, rng, "int8")
    Cg = Guarded(rows, N, dtype, ld=N + 3, band=band).set(Ch)
    Pg = Guarded(rows, N, dtype, ld=N + 5, band=band).set(Ph)
    ops.spmm_tile_accumulate(Cg.view, Pg.view)
    torch.cuda.synchronize()
    assert Cg.canaries_intact() and Pg.unchanged()
    # small integers: the sum is exact in FP32 and in BF16
    assert np.array_equal(G.host_f32(Cg.view), Ch + Ph)


@pytest.mark.parametrize("band", [64, 1])
def test_spgemm_guard_bands(band):
    G.note("canary spgemm band=%d" % band)
    rng = _rng(7)
    K, N = 3000, 20000
    L = rng.integers(0, 40, size=K)
    L[rng.choice(K, size=5, replace=False)] = [9000, 4100, 1000, 300, 129]
    B = synth.random_csr(K, N, L, rng, "int8")
    A = synth.random_csr(2000, K, rng.integers(0, 12, size=2000), rng, "int8")
    plan = ops.spgemm_create(A.rows, G.to_dev(A), G.to_dev(B), validate=True)
    rpg = Guarded(1, A.rows + 1, torch.int32, band=band)
    cig = Guarded(1, plan.nnz_c, torch.int32, band=band)
    vag = Guarded(1, plan.nnz_c, torch.float32, band=band)
    ops.spgemm_rowptr(plan, rpg.view[0])
    ops.spgemm_compute(plan, cig.view[0], vag.view[0])
    torch.cuda.synchronize()
    assert rpg.canaries_intact() and cig.canaries_intact() and vag.canaries_intact()
    r_rp, r_ci, r_va, _ = oracle.spgemm((A.rowptr, A.colind, A.values), (B.rowptr, B.colind, B.values), N)
    assert np.array_equal(rpg.view[0].cpu().numpy().astype(np.int64), r_rp)
    assert np.array_equal(cig.view[0].cpu().numpy().astype(np.int64), r_ci)
    assert np.array_equal(vag.view[0].cpu().numpy().astype(np.float64), r_va)
