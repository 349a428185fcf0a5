"""The measured summaries under profiles/ stay consistent with the code:
every committed bench line carries the fields of the bench contract, every
bench.py command quoted in a profile summary parses with the current
command line, and traffic records name a kernel id and byte counts."""

import json
import os
import re
import shlex
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
FIELDS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
          "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline",
          "cpu_baseline")


def _lines():
    for name in sorted(os.listdir(PROFILES)):
        if name.endswith(".json"):
            with open(os.path.join(PROFILES, name)) as f:
                yield name, json.loads(f.read().strip().splitlines()[-1])


@pytest.mark.parametrize("name,line", list(_lines()), ids=lambda v: v if isinstance(v, str) else "")
def test_bench_lines_follow_the_contract(name, line):
    for k in FIELDS:
        assert k in line, (name, k)
    assert line["n_gpus"] == 1 and line["value"] > 0 and line["ms_per_step"] > 0
    assert "workload" in line["config"]
    cpu = line["cpu_baseline"]
    if cpu is not None:
        assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["value"] > 0
    roof = line["roofline"]
    if roof is not None:
        assert roof["bound"] == "alu" and 0 < roof["frac"] < 1
        assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-9


def test_quoted_bench_commands_parse():
    sys.path.insert(0, ROOT)
    import bench
    found = 0
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        text = open(os.path.join(PROFILES, name)).read().replace("\\\n", " ")
        for m in re.finditer(r"bench\.py((?: +--?[\w-]+(?: +(?:'[^']*'|[^\s)(;-][^\s);]*))?)*)", text):
            argv = shlex.split(m.group(1))
            old = sys.argv
            try:
                sys.argv = ["bench.py"] + argv
                bench.parse()
            finally:
                sys.argv = old
            found += 1
    assert found >= 5


def test_traffic_records_name_kernel_and_bytes():
    recs = 0
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)):
            if line.startswith("<!-- traffic "):
                rec = json.loads(line.strip()[len("<!-- traffic "):-len("-->")])
                assert re.fullmatch(r"[0-9a-f]{16}", rec["kernel_id"])
                assert rec["fetch_bytes"] > 0 and rec["write_bytes"] > 0
                recs += 1
    assert recs >= 1
