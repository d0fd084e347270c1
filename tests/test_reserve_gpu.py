"""Reservation-grid hand-out (the work grids of the work-stealing algorithms, Algorithm 3, on one
GPU): the stationary-A step of a tile row, C(0,j) += sum_k A(0,k) B(k,j), computed as a batch of
component products into partial tiles and drained in k order by the owner's accumulate, against
the FP64 oracle; every grid mode against the others and against one launch per product."""
import numpy as np
import pytest
import torch

import synth
from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu

MODES = ["2d", "3d", "own"]


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _tile_row(seed, M=3000, K=3, J=3, value_kind="int8", long_rows=True):
    rng = _rng(seed)
    As = []
    for k in range(K):
        cols = int(rng.integers(500, 2500))
        L = rng.integers(0, 25 if k == 0 else 6, size=M)      # k-tiles of very different weight
        if long_rows:
            L[rng.integers(0, M, size=3)] = min(cols, 700)
        As.append(synth.random_csr(M, cols, L, rng, value_kind))
    Ns = [int(n) for n in rng.choice([32, 64, 128], size=J)]
    Bs = [[synth.dense(A.cols, Ns[j], rng, value_kind) for j in range(J)] for A in As]
    C0 = [synth.dense(M, Ns[j], rng, value_kind) for j in range(J)]
    return As, Ns, Bs, C0


def _stationary_a(handles, As, Ns, Bs, C0, mode, dtype=torch.float32, reps=1):
    K, J = len(As), len(Ns)
    tiles, tN, coords, Bd, Pd = [], [], [], [], []
    for k in range(K):
        for j in range(J):
            tiles.append(handles[k])
            tN.append(Ns[j])
            coords.append((0, j, k))
            Bd.append(G.dense_dev(Bs[k][j], dtype))
            Pd.append(torch.empty(As[k].rows, Ns[j], dtype=dtype, device=G.DEV))
    batch = ops.spmm_batch_create_grid(tiles, tN, coords, mode, dtype) if mode != "loop" else None
    Cs = None
    for _ in range(reps):
        Cs = [G.dense_dev(c, dtype) for c in C0]
        if batch is None:
            for t in range(len(tiles)):
                ops.spmm_fwd(tiles[t], [Bd[t]], C=Pd[t])
        else:
            ops.spmm_batched(batch, Bd, Pd)
        for j in range(J):
            ops.spmm_tile_accumulate_n(Cs[j], [Pd[k * J + j] for k in range(K)])
    torch.cuda.synchronize()
    return Cs


@pytest.mark.parametrize("mode", MODES)
def test_stationary_a_grid_integer_exact(mode):
    G.note("reserve grid integer mode=%s" % mode)
    As, Ns, Bs, C0 = _tile_row(1)
    handles = [G.make_tile([A], long_row=128, segment=64) for A in As]
    assert handles[0].stats()["long_rows"] > 0
    Cs = _stationary_a(handles, As, Ns, Bs, C0, mode, reps=2)
    for j in range(len(Ns)):
        ref, _ = G.oracle_fwd(As, [Bs[k][j] for k in range(len(As))], accumulate=True, C0=C0[j])
        assert np.array_equal(G.host_f32(Cs[j]).astype(np.float64), ref), (mode, j)


def test_stationary_a_grid_modes_agree_fp32():
    """Real-valued data: every grid mode and the per-product launch loop give the same bits (each item
    is summed by one wave in CSR order, split rows in unit order, partials drained in k order), and
    match the oracle within the FP32 bound."""
    G.note("reserve grid modes agree")
    As, Ns, Bs, C0 = _tile_row(2, value_kind="pm1")
    handles = [G.make_tile([A], long_row=128, segment=64) for A in As]
    ref_C = _stationary_a(handles, As, Ns, Bs, C0, "loop")
    for mode in MODES:
        Cs = _stationary_a(handles, As, Ns, Bs, C0, mode)
        for j in range(len(Ns)):
            assert torch.equal(Cs[j], ref_C[j]), (mode, j)
    for j in range(len(Ns)):
        ref, S = G.oracle_fwd(As, [Bs[k][j] for k in range(len(As))], accumulate=True, C0=C0[j])
        n = G.row_terms(As) + 1 + len(As)
        G.assert_fp32_close(G.host_f32(ref_C[j]), ref, S + np.abs(C0[j]), n, what="C(0,%d)" % j)


@pytest.mark.parametrize("mode", MODES)
def test_stationary_a_grid_bf16(mode):
    G.note("reserve grid bf16 mode=%s" % mode)
    As, Ns, Bs, C0 = _tile_row(3, value_kind="pm1", long_rows=False)
    handles = [G.make_tile([A]) for A in As]
    ref_C = _stationary_a(handles, As, Ns, Bs, C0, "loop", dtype=torch.bfloat16)
    Cs = _stationary_a(handles, As, Ns, Bs, C0, mode, dtype=torch.bfloat16)
    for j in range(len(Ns)):
        assert torch.equal(Cs[j], ref_C[j]), (mode, j)


def test_grid_many_entries_and_graph_replay():
    """More entries than XCDs (a 2 x 3 x 4 grid), every mode; the 3-D mode captured in a graph and
    replayed (the reset kernel rearms the counters)."""
    G.note("reserve grid many entries")
    rng = _rng(5)
    I, J, K, M = 2, 3, 4, 700
    A = {(i, k): synth.random_csr(M, 400 + 50 * k, rng.integers(0, 12, size=M), rng, "int8")
         for i in range(I) for k in range(K)}
    H = {ik: G.make_tile([a]) for ik, a in A.items()}
    N = 64
    B = {(k, j): synth.dense(400 + 50 * k, N, rng, "int8") for k in range(K) for j in range(J)}
    tiles, coords, Bd, keys = [], [], [], []
    for i in range(I):
        for j in range(J):
            for k in range(K):
                tiles.append(H[(i, k)])
                coords.append((i, j, k))
                Bd.append(G.dense_dev(B[(k, j)]))
                keys.append((i, j, k))
    want = {}
    for (i, j, k) in keys:
        ref, _ = G.oracle_fwd([A[(i, k)]], [B[(k, j)]])
        want[(i, j, k)] = ref
    for mode in MODES:
        batch = ops.spmm_batch_create_grid(tiles, [N] * len(tiles), coords, mode)
        Pd = [torch.full((M, N), float("nan"), device=G.DEV) for _ in tiles]
        ops.spmm_batched(batch, Bd, Pd)
        torch.cuda.synchronize()
        for t, key in enumerate(keys):
            assert np.array_equal(G.host_f32(Pd[t]).astype(np.float64), want[key]), (mode, key)
        if mode != "3d":
            continue
        ws = batch.workspace()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            ops.spmm_batched(batch, Bd, Pd, workspace=ws)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ops.spmm_batched(batch, Bd, Pd, workspace=ws)
        for r in range(5):
            for p in Pd:
                p.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            for t, key in enumerate(keys):
                assert np.array_equal(G.host_f32(Pd[t]).astype(np.float64), want[key]), (r, key)


def test_accumulate_n_order_and_many_partials():
    """C += P_0 + ... + P_{n-1} in order, more partials than one launch takes (integer data: exact;
    BF16: the FP32 sum of each group of 16 rounded once)."""
    G.note("accumulate_n")
    rng = _rng(6)
    rows, N, n = 300, 40, 37
    C0 = synth.dense(rows, N, rng, "int8")
    Ps = [synth.dense(rows, N, rng, "int8") for _ in range(n)]
    C = G.dense_dev(C0)
    ops.spmm_tile_accumulate_n(C, [G.dense_dev(p) for p in Ps])
    torch.cuda.synchronize()
    want = C0.astype(np.float64) + sum(p.astype(np.float64) for p in Ps)
    assert np.array_equal(G.host_f32(C).astype(np.float64), want)
