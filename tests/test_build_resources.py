"""Kernel resource use of the built library (compiler remarks recorded by the
build): no kernel may use scratch memory, spill registers or need a dynamic
stack.  A device function that is not inlined into its kernel becomes a call
with a stack in scratch memory, whose traffic and call overhead land in the
hot loops (the shared tile functions of the squaring, the chain application
and the score are forced inline for this reason)."""

import json
import os

import pytest

from paper_1802_05421_amd import _build

HOT = ("k_square", "k_apply_gemm", "k_score", "k_residual_gemm", "k_gram_dist", "k_rhs",
       "k_exp_sym", "k_normalize")


def _resources():
    if not os.path.exists(_build.RESOURCES) or not os.path.exists(_build.LIB):
        pytest.skip("library not built")
    newest = max(os.path.getmtime(p) for p in _build.sources())
    if os.path.getmtime(_build.RESOURCES) < newest:
        pytest.skip("library built before the last source change; rebuild first")
    with open(_build.RESOURCES) as f:
        return json.load(f)


def test_remarks_parse():
    text = ("x.hip:1:1: remark: Function Name: _Z3fooPd [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     VGPRs: 12 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     Dynamic Stack: True [-Rpass-analysis=kernel-resource-usage]\n")
    assert _build.parse_resources(text) == {"_Z3fooPd": {"vgpr": 12, "scratch": 16,
                                                         "dynamic_stack": True}}


def test_no_kernel_uses_scratch_or_spills():
    res = _resources()
    assert len(res) > 50
    bad = {k: v for k, v in res.items()
           if v.get("scratch", 0) or v.get("vgpr_spill", 0) or v.get("sgpr_spill", 0)
           or v.get("dynamic_stack", False)}
    assert not bad, bad


def test_hot_kernels_present_and_resident():
    res = _resources()
    for h in HOT:
        ks = [v for k, v in res.items() if h in k]
        assert ks, h
        for v in ks:
            assert v["occupancy"] >= 1 and v["vgpr"] + v.get("agpr", 0) <= 512, (h, v)
