"""Entry points with roctx ranges switched on (SPMM_TRACE=1, read once per process, so in a
child process): forward, backward, batch and SpGEMM still match the oracle."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = r'''
import sys
sys.path.insert(0, "tests")
import numpy as np, torch
import synth, oracle
import gpu_util as G
from paper_2311_18141_amd import ops
rng = np.random.Generator(np.random.PCG64(61))
A = synth.random_csr(700, 500, rng.integers(0, 40, size=700), rng, "int8")
B = synth.dense(A.cols, 64, rng, "int8")
dC = synth.dense(A.rows, 64, rng, "int8")
t = G.make_tile([A], transpose=True)
C = G.fwd(t, [G.dense_dev(B)])
ref, _ = G.oracle_fwd([A], [B])
assert np.array_equal(G.host_f32(C).astype(np.float64), ref)
dA, dB = ops.spmm_bwd(t, G.dense_dev(dC), G.dense_dev(B))
torch.cuda.synchronize()
assert np.array_equal(dA.cpu().numpy().astype(np.float64), oracle.sddmm(A.rowptr, A.colind, dC, B)[0])
assert np.array_equal(G.host_f32(dB).astype(np.float64), oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)[0])
batch = ops.spmm_batch_create([G.make_tile([A])], [64])
Cb = torch.empty(A.rows, 64, device=G.DEV)
ops.spmm_batched(batch, [G.dense_dev(B)], [Cb])
torch.cuda.synchronize()
assert np.array_equal(G.host_f32(Cb).astype(np.float64), ref)
S = synth.random_csr(500, 300, rng.integers(0, 10, size=500), rng, "int8")
plan = ops.spgemm_create(A.rows, G.to_dev(A), G.to_dev(S))
ci, va = ops.spgemm_compute(plan)
torch.cuda.synchronize()
r_rp, r_ci, r_va, _ = oracle.spgemm((A.rowptr, A.colind, A.values), (S.rowptr, S.colind, S.values), S.cols)
assert np.array_equal(ci.cpu().numpy().astype(np.int64), r_ci) and np.array_equal(va.cpu().numpy().astype(np.float64), r_va)
print("ok")
'''


def test_entry_points_with_trace_ranges():
    env = dict(os.environ, SPMM_TRACE="1")
    r = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-3000:])
