"""The library called with PyTorch device memory and a PyTorch stream.

PyTorch-ROCm ships its own HIP runtime, whose shared object carries the same
soname (libamdhip64.so.7) as the ROCm runtime the library is linked against.
A process that imports torch first therefore has that runtime loaded when the
library is opened, and the dynamic linker binds the library to it: one HIP
runtime in the process, so torch tensors are valid device pointers for the
library and torch streams are valid streams.  The test runs in a fresh
process (the pytest process may already hold the library on the ROCm
runtime), checks that exactly one libamdhip64 is mapped, and compares the
results with Table 1 and with oracle values.
"""
import json
import os
import subprocess
import sys

import pytest

from conftest import GOLDEN, ROOT, read_table

CHILD = r"""
import json, sys
import torch                                   # first: its HIP runtime is the process's
assert torch.cuda.is_available()
sys.path.insert(0, sys.argv[1])
import paper_1503_01839_amd as pc
pc.lib()
xs = json.loads(sys.argv[2])
hips = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})
dev = torch.device('cuda', 0)
n = len(xs)
d_xs = torch.tensor(xs, dtype=torch.int64, device=dev)   # every x < 2^63
d_out = torch.full((n,), -1, dtype=torch.int64, device=dev)
wsb = pc.workspace_bytes(xs)
d_ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
s = torch.cuda.Stream(device=dev)              # default priority
with torch.cuda.stream(s):
    d_xs2 = d_xs.flip(0).contiguous()         # torch work queued on the same stream first
    d_out2 = torch.full((n,), -1, dtype=torch.int64, device=dev)
    pc.pi_count_batch_async(d_xs, n, d_out, d_ws, wsb, stream=torch.cuda.current_stream())
    pc.pi_count_batch_async(d_xs2, n, d_out2, d_ws, wsb, stream=torch.cuda.current_stream())
    tot = d_out.sum()                         # torch work that reads the library's output
s.synchronize()
print(json.dumps({"hip": hips, "out": d_out.cpu().tolist(), "out2": d_out2.cpu().tolist(),
                  "sum": int(tot.item()), "solo": [pc.pi_count(x) for x in xs[:6]]}))
"""


@pytest.mark.gpu
def test_torch_tensors_and_stream(paper_pow10):
    mixes = json.load(open(os.path.join(GOLDEN, "oracle_pi_mixes.json")))
    want = {n_: v for n_, v in mixes["serve_test"][:40]}
    want.update({10**k: paper_pow10[k] for k in range(1, 17)})
    want.update({1: 0, 2: 1, 3: 2, 0: 0})
    xs = sorted(want)
    print("step: torch child process", len(xs), "queries", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(xs)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert len(got["hip"]) == 1, f"more than one HIP runtime mapped: {got['hip']}"
    assert "torch" in got["hip"][0], got["hip"]
    assert got["out"] == [want[x] for x in xs]
    assert got["out2"] == [want[x] for x in reversed(xs)]
    assert got["sum"] == sum(want.values())
    assert got["solo"] == [want[x] for x in xs[:6]]
