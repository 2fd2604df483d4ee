"""The C ABI from a plain C program (tests/c_abi/consumer.c, built by
__graft_entry__.build()): the HIP runtime for device memory and a stream,
libqmc.so for the work, no Python binding or torch in between.  Its printed
results against the FP64 oracle, to the bars of the other parity tests."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2404_08867_amd", "_build", "qmc_c_consumer")


def test_plain_c_consumer_matches_oracle():
    assert os.path.exists(EXE), "build the C consumer first (__graft_entry__.build())"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    out = {ln.split()[0]: ln.split()[1:] for ln in r.stdout.splitlines() if ln.strip()}
    z = O.korobov(4, 1009, 76)
    assert [int(v) for v in out["korobov"]] == [int(v) for v in z]
    qo, ao = O.lattice_sum(z, 1009, O.EXP_SUM, np.array([0.3, 0.6, 0.9, 1.2]))
    for name, tol in (("lattice_sum_fp64", 1e-12), ("lattice_sum_fp32c", 1e-6)):
        q = float(out[name][0])
        assert abs(q - qo) <= tol * max(abs(qo), ao), (name, q, qo)
    mo = O.mdi_lr(np.array([5, 6, 7]), O.GAUSSIAN, np.array([0.5, 0.8, 1.1, 0.2, 0.5, 0.7]))
    qm = float(out["mdi_lr_fp64"][0])
    assert abs(qm - mo) <= 1e-12 * abs(mo), (qm, mo)
