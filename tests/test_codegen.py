"""Host checks of the kernel generator: every schedule's passes cover each
moment component exactly once (moments, reverse sweep, adjoint), the graph
groups of the loss path cover each connected graph once, and every kernel a
launcher names is defined."""
import re

import pytest

from paper_2007_08555_amd import codegen


@pytest.mark.parametrize("level", [8, 12, 16])
def test_passes_partition_the_components(level):
    s = codegen.Schedule(level)
    comp_nu = {k: nu for (mu, nu, abc), k in s.comp.items()}
    for sch in [codegen.SCHEDULE_F32] + codegen.SCHEDULES_F64:
        # the fused schedule sums every component in one kernel
        for key in ("adj",) if sch.get("fused") else ("mom", "adj"):
            seen = [k for _, comps in codegen.adjoint_passes(s, sch[key]) for k in comps]
            assert sorted(seen) == list(range(s.C))
        if sch.get("fused"):
            continue
        groups = [tuple(n for n in g if n <= s.nu_max) for g in sch["rev"]]
        covered = [n for g in groups for n in g if any(comp_nu[k] == n for k in range(s.C))]
        assert len(covered) == len(set(covered))
    groups = codegen.graph_groups(s, 40)
    assert sorted(g for grp in groups for g in grp) == list(range(len(s.terms)))


@pytest.mark.parametrize("level", [8, 16])
def test_launched_kernels_are_defined(level):
    src, _ = codegen.generate(level)
    src = src.replace("mtp::contract_table", "contract_table")
    launched = set(re.findall(r"hipLaunchKernelGGL\(\((\w+)<", src))
    defined = set(re.findall(r"(\w+_c?kernel)\(const mtp::EvalArgs", src))
    assert launched and launched <= defined, launched - defined
    # one case per FP64 schedule in the evaluation launcher
    assert len(re.findall(r"\n\s*case \d+: \{", src)) == len(codegen.SCHEDULES_F64)


@pytest.mark.parametrize("level", [20])
def test_table_level_launches(level):
    src, meta = codegen.generate_table(level)
    launched = set(re.findall(r"hipLaunchKernelGGL\(\((?:mtp::)?(\w+)<", src))
    defined = set(re.findall(r"(\w+_c?kernel)\(const mtp::EvalArgs", src))
    defined |= {"contract_table_kernel", "contract_table_loss_kernel", "contract_table_split_kernel",
                "contract_table_loss_split_kernel"}   # csrc/contract_table.h
    defined |= {"adjoint_sums_kernel"}   # csrc/mtp_device.h
    assert launched and launched <= defined, launched - defined
    assert meta["table"] and meta["loss"] and meta["trie_nodes"] > 0
