"""The compiler's resource report of every kernel instance (written by the
build from hipcc's kernel-resource-usage remarks), checked on the CPU:

* every row-resident / split-row instance the library dispatches to, the
  multi-row LayerNorm / RMSNorm forward included, is in the report
  (registers, private bytes per lane, waves per SIMD);
* the library's register model, which sizes the persistent grid where no
  device can be asked, never promises more workgroups per CU than the
  compiled code allows;
* instances whose code uses private memory (spilled registers, stack arrays)
  are exactly the ones listed below.  Split plans of those run only at the
  per-CU count a co-residency probe verified on the device (checked on the
  GPU); a kernel change that adds or removes private memory fails here first,
  so the list and that verification stay in step."""
import json
import os
import re

import pytest

from paper_2609_01864_amd import build as B
from paper_2609_01864_amd import credit as C

VPTS = (1, 2, 4, 8, 12, 16, 24, 32, 48, 68)
# (kernel operator index, dtype index) -> public (op, direction)
KOPS = {0: (C.SOFTMAX, C.FWD), 1: (C.LAYERNORM, C.FWD), 2: (C.RMSNORM, C.FWD), 3: (C.SOFTMAX, C.BWD),
        4: (C.LAYERNORM, C.BWD), 5: (C.RMSNORM, C.BWD), 6: (C.SOFTMAX_LOGITS, C.BWD), 7: (C.QUANT_INT8, C.FWD),
        8: (C.QUANT_FP8, C.FWD), 9: (C.PEARSON, C.BWD), 10: (C.WVAR, C.BWD), 11: (C.LAYERNORM_FP8_OUT, C.FWD)}
ROWS = (1, 2, 4)
# (kernel operator, dtype, vectors per thread, rows per workgroup) of the
# instances with private memory
PRIVATE = {(0, 0, 16, 1), (0, 0, 24, 1), (0, 0, 48, 1), (0, 1, 16, 1), (0, 1, 24, 1), (0, 1, 48, 1), (1, 2, 12, 1),
           (4, 0, 4, 1), (4, 0, 8, 1), (4, 1, 1, 1), (4, 1, 2, 1), (4, 1, 4, 1), (4, 2, 1, 1), (4, 2, 2, 1),
           (5, 1, 2, 1), (5, 2, 2, 1), (5, 2, 4, 1), (6, 2, 1, 1), (6, 2, 2, 1), (6, 2, 4, 1), (11, 1, 32, 1)}


@pytest.fixture(scope="module")
def report(lib_built):
    if not os.path.exists(B.RESOURCES):
        B.build(verbose=False)
    with open(B.RESOURCES) as f:
        rep = json.load(f)
    out = {}
    for name, r in rep.items():
        # k_resident<op, dtype, register vectors, LDS vectors>: keyed by the
        # slice bucket (register + LDS vectors per thread)
        m = re.fullmatch(r"_ZN6credit10k_residentILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)EEEvNS_7RowArgsE", name)
        if m:
            op, dt, v, lds = (int(g) for g in m.groups())
            out[(op, dt, v + lds, 1)] = r
        # k_multirow<op, dtype, vectors, rows>
        m = re.fullmatch(r"_ZN6credit10k_multirowILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)EEEvNS_7RowArgsE", name)
        if m:
            op, dt, v, rows = (int(g) for g in m.groups())
            out[(op, dt, v, rows)] = r
    return out


def _dispatched():
    for kop, (o, d) in KOPS.items():
        for dt in (C.F32, C.BF16, C.FP8):
            for v in VPTS:
                for rows in ROWS:
                    try:
                        info = C.instance_info(None, o, d, dt, v, rows)
                    except C.CreditError:  # no such (operator, dtype)
                        continue
                    if info is not None:
                        yield (kop, dt, v, rows), info


def test_every_dispatched_instance_is_reported(report):
    seen = 0
    for key, _ in _dispatched():
        assert key in report, key
        r = report[key]
        assert {"vgprs", "scratch_bytes", "waves_per_simd"} <= set(r), key
        seen += 1
    assert seen == len(report) > 190


def test_register_model_is_a_lower_bound(report):
    # one workgroup is one wave per SIMD, so waves per SIMD = workgroups per CU
    for key, info in _dispatched():
        assert info["model_per_cu"] <= report[key]["waves_per_simd"], (key, info, report[key])


def test_instances_with_private_memory(report):
    private = {k for k, r in report.items() if r["scratch_bytes"] > 0}
    assert private == PRIVATE, f"added: {sorted(private - PRIVATE)}, gone: {sorted(PRIVATE - private)}"
