"""Allocation failures on a device: every partial-allocation path of the
create calls returns PWFS_ERR_OUT_OF_MEMORY and gives back what it had
allocated.

Runs in a fresh child process (the allocation fault hook reads
PWFS_FAULT_INJECT at each device allocation; "oom:N" fails the N-th one after
the variable took that value).  The child creates and destroys one plan and
one network first (so that the runtime's own lazily made buffers exist), takes
the device's free memory, then for N = 1, 2, ... fails the N-th allocation of
pwfs_plan (LBT-like geometry, 4 frames: ~41 MB of row-pass workspace) and of
pwfs_cnn_create until a call succeeds, destroys that one, and compares the free
memory with the baseline.
"""
import json
import os
import subprocess
import sys

import pytest

from tests.gpu_common import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes, json, os, sys
sys.path.insert(0, %r)
import torch
import paper_1607_07624_amd as pw
from paper_1607_07624_amd._lib import make_config
from paper_1607_07624_amd.cnn import cnn_config, _lib as cnn_lib
from synth.configs import CFG2
torch.cuda.init()
lib = pw.load_library()
clib = cnn_lib()

def plan(batch):
    h = ctypes.c_void_p()
    st = lib.pwfs_plan(ctypes.byref(make_config(CFG2, batch)), None, ctypes.byref(h))
    return st, h

def net():
    h = ctypes.c_void_p()
    c = cnn_config(n_sub=40, c1=32, c2=64, c3=64, hidden=2048, n_out=600, batch_max=64, reserved=0)
    return clib.pwfs_cnn_create(ctypes.byref(c), ctypes.byref(h)), h

st, h = plan(4); assert st == 0; lib.pwfs_destroy(h)
st, h = net(); assert st == 0; clib.pwfs_cnn_destroy(h)
torch.cuda.synchronize()
free0 = torch.cuda.mem_get_info()[0]
out = {}
for name, make, destroy in (("plan", lambda: plan(4), lib.pwfs_destroy), ("cnn", net, clib.pwfs_cnn_destroy)):
    statuses = []
    for n in range(1, 200):
        os.environ["PWFS_FAULT_INJECT"] = "oom:%%d" %% n
        st, h = make()
        statuses.append(st)
        if st == 0:
            destroy(h)
            break
        assert not h.value, "handle set on failure"
    os.environ.pop("PWFS_FAULT_INJECT")
    out[name] = statuses
torch.cuda.synchronize()
out["leaked_bytes"] = int(free0 - torch.cuda.mem_get_info()[0])
print(json.dumps(out), flush=True)
''' % ROOT


def test_allocation_failures_return_oom_and_leak_nothing():
    env = {k: v for k, v in os.environ.items() if k != "PWFS_FAULT_INJECT"}
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    res = json.loads(r.stdout.strip().splitlines()[-1])
    say(f"[gpu] fault injection: plan statuses {res['plan']}, cnn statuses {res['cnn']}, "
        f"free memory change {res['leaked_bytes']} B")
    for name in ("plan", "cnn"):
        st = res[name]
        assert st[-1] == 0 and len(st) >= 5, name                # several allocations, then success
        assert all(s == -4 for s in st[:-1]), name               # PWFS_ERR_OUT_OF_MEMORY each time
    assert abs(res["leaked_bytes"]) <= 4 << 20                   # within the runtime's granularity
