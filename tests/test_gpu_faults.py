"""Error paths forced from the host: RSB_FAULT_INJECT makes the N-th device
allocation or the N-th launch check of a call fail.  Every such call must
return RSB_EDEVICE with the injected message, leave nothing behind that
changes a later call (same partition afterwards) and not grow the device
memory in use over repeated failures.  A memory limit below what a call
needs gives RSB_ENOMEM, and the restart cap gives a warning with a valid
partition.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb

pytestmark = pytest.mark.gpu

MESH = mg.uniform_holes(mg.box_hex(12, 10, 8), 0.05, 1)


@pytest.mark.parametrize("spec", ["alloc:1", "alloc:7", "alloc:40", "launch:1", "launch:25",
                                  "launch:60"])
def test_injected_failure_reports_and_recovers(monkeypatch, spec):
    import torch
    st0, p0, _ = rsb.partition(MESH.ids, 8, tol=1e-6)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        monkeypatch.setenv("RSB_FAULT_INJECT", spec)
        with pytest.raises(rsb.RsbError) as e:
            rsb.partition(MESH.ids, 8, tol=1e-6)
        assert e.value.code == rsb.EDEVICE and "injected" in str(e.value)
        monkeypatch.delenv("RSB_FAULT_INJECT")
    st, p, _ = rsb.partition(MESH.ids, 8, tol=1e-6)
    assert st == st0 and np.array_equal(p, p0)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)


def test_memory_limit_and_restart_cap():
    with pytest.raises(rsb.RsbError) as e:
        rsb.partition(MESH.ids, 8, device_mem_limit=1 << 16)
    assert e.value.code == rsb.ENOMEM
    st, part, stats = rsb.partition(MESH.ids, 8, lanczos_m=2, max_restarts=0)
    # a warning (2, a disconnected subgraph, outranks 1) and unconverged solves
    assert st in (1, 2) and stats["not_converged"] > 0
    sizes = np.bincount(part, minlength=8)
    assert sizes.max() - sizes.min() <= 1
