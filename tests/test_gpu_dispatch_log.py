"""HDC_LOG=1 on the device entry points: every call prints its dispatch
decision (one line on stderr), and the decision named is the one the tuning
selects.  The switch is read once per process, so the calls run in one child
process; their results are checked there against plain torch references."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import torch, paper_2309_03912_amd as hdc
dev = torch.device("cuda", 0)
x = torch.linspace(-1, 1, 4099, device=dev)
y = torch.empty_like(x)
hdc.map(x, hdc.affine(2.5, 0.5), out=y)
assert torch.equal(y, (2.5 * x.double() + 0.5).float())
ym = torch.empty(4100, device=dev)
hdc.map(x[1:], hdc.identity(), out=ym[:4098])   # x and y misaligned by 4 bytes mod 16
assert torch.equal(ym[:4098], x[1:])
r = hdc.transform_reduce(x, hdc.identity(), "compensated")
assert abs(float(r) - float(x.double().sum())) < 1e-9
hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, 0, block=256, unroll=2, grid_mult=2, passes=1)
r = hdc.transform_reduce(x, hdc.identity(), "plain")
assert abs(float(r) - float(x.double().sum())) < 1e-3
r = hdc.transform_reduce_noalloc(x, hdc.identity(), "compensated")
assert abs(float(r) - float(x.double().sum())) < 1e-9
z = torch.ones_like(x)
r = hdc.transform_reduce(x, hdc.product(), "plain", z=z)
off = torch.tensor([0, 10, 10, 4000, 4099], dtype=torch.int64, device=dev)
s = hdc.segmented_reduce(x, off, hdc.identity(), "compensated")
ref = torch.stack([x[a:b].double().sum() for a, b in zip(off[:-1].tolist(), off[1:].tolist())])
assert torch.allclose(s, ref, atol=1e-9)
p = hdc.scan(x, hdc.identity(), "compensated")
assert torch.allclose(p, x.double().cumsum(0), atol=1e-9)
q = hdc.segmented_scan(x, off, hdc.identity(), "compensated", exclusive=True)
torch.cuda.synchronize()
print("child ok")
"""


@pytest.mark.gpu
def test_dispatch_log_lines():
    env = dict(os.environ, HDC_LOG="1")
    p = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert p.returncode == 0 and "child ok" in p.stdout, p.stderr[-3000:]
    lines = [l for l in p.stderr.splitlines() if l.startswith("hdc: ")]

    def has(prefix, *parts):
        return any(l.startswith("hdc: " + prefix) and all(s in l for s in parts) for l in lines)

    assert has("map dtype=f32 acc=plain n=4099 ", "schedule=16-byte vectors", "workspace=none"), lines
    assert has("map dtype=f32 acc=plain n=4098 ", "schedule=scalar (x, y misaligned)"), lines
    # the binding passes a workspace of its own: the library logs it as the caller's
    assert has("transform_reduce dtype=f32 acc=compensated n=4099 ", "workspace=caller"), lines
    assert has("transform_reduce dtype=f32 acc=plain n=4099 bucket=0 block=256 unroll=2 grid_mult=2",
               "passes=1", "schedule=one launch (the last block folds the partials)"), lines
    assert has("transform_reduce dtype=f32 acc=compensated n=4099 ", "workspace=static scratch"), lines
    assert has("dot dtype=f32 acc=plain n=4099 "), lines
    assert has("segmented_reduce dtype=f32 acc=compensated ", "schedule=t") or \
        has("segmented_reduce dtype=f32 acc=compensated ", "schedule=planned"), lines
    assert has("scan (inclusive) dtype=f32 acc=compensated n=4099 ", "schedule="), lines
    assert has("segmented_scan (exclusive) dtype=f32 acc=compensated n=4099 ", "schedule="), lines
