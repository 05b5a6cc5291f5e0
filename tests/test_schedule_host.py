"""The library's host-side schedule tables (built without a GPU) against the oracle: the
forward run lists of every memory mode and reading, and their transpose for the adjoint's
reverse sweep (offset m of reverse step rho = n - 1 - k weighted by its multiplicity in the
schedule of forward step k + m), which the oracle's adjoint forms by scattering each
step's terms.  Built from the library's sources with hipcc as a host-only program."""
import os
import shutil
import subprocess
from collections import defaultdict

import pytest

import oracle
from paper_1004_5128_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODES = {"full": 0, "short": 1, "adaptive": 2}
RULES = {"partition": 0, "literal": 1, "unit_stride": 2}


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("sched") / "schedule_probe")
    csrc = os.path.join(ROOT, "paper_1004_5128_amd", "csrc")
    subprocess.run([hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "host", "schedule_probe.cpp"),
                    os.path.join(csrc, "gl_schedule.cpp"), "-o", exe], check=True,
                   capture_output=True)
    return exe


def run_probe(exe, mem, n):
    out = subprocess.run([exe, str(MODES[mem["mode"]]), str(RULES[mem["rule"]]), str(mem["L"]),
                          str(mem["a"]), str(n)], check=True, capture_output=True, text=True)
    tables = {"F": {}, "T": {}}
    for line in out.stdout.splitlines():
        kind, k, terms, *runs = line.split()
        terms_of = defaultdict(int)
        seq = []
        for r in runs:
            m0, cnt, stride, coef = map(int, r.split(":"))
            for t in range(cnt):
                terms_of[m0 + t * stride] += coef
                seq.append(m0 + t * stride)
        assert len(seq) == int(terms)
        tables[kind][int(k)] = (dict(terms_of), seq)
    return tables


MEMS = [W.memory("full"), W.memory("short", L=7), W.memory("adaptive", a=2),
        W.memory("adaptive", a=3), W.memory("adaptive", a=3, rule="literal"),
        W.memory("adaptive", a=4, rule="literal"), W.memory("adaptive", a=2, rule="unit_stride")]


@pytest.mark.parametrize("mem", MEMS, ids=lambda m: "%s-%s-%d-%d" % (m["mode"], m["rule"], m["L"], m["a"]))
def test_forward_and_transposed_schedules_match_oracle(probe, mem):
    n = 400
    tables = run_probe(probe, mem, n)
    trans = defaultdict(lambda: defaultdict(float))
    for k in range(n):
        ms, cs = oracle.schedule(mem, k)
        got, seq = tables["F"][k]
        assert got == {int(m): int(c) for m, c in zip(ms, cs)}, k
        for m, c in zip(ms, cs):
            trans[n - 1 - (k - int(m))][int(m)] += c
    for rho in range(n):
        got, seq = tables["T"][rho]
        assert got == {m: int(c) for m, c in trans[rho].items()}, rho
        assert seq == sorted(seq) and seq[0] == 0 and got[0] == 1   # ascending, m = 0 first
        if mem["mode"] != "adaptive":   # full and short memory are their own transposes
            assert got == tables["F"][rho][0], rho


def test_random_settings_match_oracle(probe):
    # seeded random memory settings and run lengths, forward and transposed tables
    import numpy as np
    rng = np.random.default_rng(77)
    for _ in range(24):
        mode = ["full", "short", "adaptive"][int(rng.integers(3))]
        mem = W.memory(mode, L=int(rng.integers(0, 60)), a=int(rng.integers(2, 9)),
                       rule=["partition", "literal", "unit_stride"][int(rng.integers(3))])
        n = int(rng.integers(1, 260))
        tables = run_probe(probe, mem, n)
        trans = defaultdict(lambda: defaultdict(float))
        for k in range(n):
            ms, cs = oracle.schedule(mem, k)
            assert tables["F"][k][0] == {int(m): int(c) for m, c in zip(ms, cs)}, (mem, n, k)
            for m, c in zip(ms, cs):
                trans[n - 1 - (k - int(m))][int(m)] += c
        for rho in range(n):
            assert tables["T"][rho][0] == {m: int(c) for m, c in trans[rho].items()}, (mem, n, rho)
