"""CPU-side checks of the product's host logic and of the C-ABI library (no GPU).

* The library loads and exports every function declared in include/rmc.h.
* The product-side term lists (spin_models) reproduce the oracle's dense model
  Hamiltonians bit for bit when assembled in list order (the same accumulation
  order the leaf kernel uses).
* The seeded workload generators are deterministic and have the stated shapes.
"""
import os
import re
from functools import reduce

import numpy as np
import pytest

from oracle import hamiltonian as OH
from paper_2609_02394_amd import spin_models as SM
from paper_2609_02394_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_P = {"I": np.eye(2), "X": np.array([[0.0, 1.0], [1.0, 0.0]]),
      "T": np.array([[0.0, -1.0], [1.0, 0.0]]), "Z": np.array([[1.0, 0.0], [0.0, -1.0]])}


def _dense(n, terms):
    H = np.zeros((2 ** n, 2 ** n))
    for c, ops in terms:
        d = dict(ops)
        H = H + c * reduce(np.kron, [_P[d.get(i, "I")] for i in range(n)])
    return H


def header_functions():
    src = open(os.path.join(ROOT, "include", "rmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rmc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_calls():
    f = header_functions()
    for name in ("rmc_module_ed", "rmc_project_ops", "rmc_couple_solve", "rmc_recurse"):
        assert name in f


def test_library_exports_every_declared_symbol():
    import ctypes

    from paper_2609_02394_amd import rmc

    if not os.path.exists(rmc.LIB_PATH):
        pytest.skip("librmc.so not built")
    lib = ctypes.CDLL(rmc.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(rmc.EXPORTED)
    rmc.load_library()  # signatures bind


def test_default_opts_without_gpu():
    from paper_2609_02394_amd import rmc

    if not os.path.exists(rmc.LIB_PATH):
        pytest.skip("librmc.so not built")
    o = rmc.default_opts()
    assert o.precision == rmc.FP64 and o.tol == 1e-13 and o.gap_tol == 1e-6


def test_job_batch_marshals_each_job_once():
    """A JobBatch holds one descriptor per job with the chain's fields and its terms,
    site by site and operator by operator, as make_terms writes them."""
    from paper_2609_02394_amd import rmc

    jobs = [rmc.job_chain(j) for j in W.rfheis_batch(6)] + [rmc.job_chain(W.tfim_small())]
    b = rmc.JobBatch(jobs)
    assert len(b) == 7 and b.qmax == max(j[4] for j in jobs)
    for d, (ns, ls, terms, k, q) in zip(b.descs, jobs):
        assert not d.tree and d.chain
        c = d.chain.contents
        assert (c.n_sites, c.leaf_sites, c.n_terms, c.k, c.q) == (ns, ls, len(terms), k, q)
        for t, (coef, ops) in enumerate(terms):
            tm = c.terms[t]
            assert tm.coef == coef and tm.nsite == len(ops)
            assert [(tm.site[u], tm.op[u]) for u in range(len(ops))] == \
                [(s, rmc.OPS[o]) for s, o in ops]


@pytest.mark.parametrize("job", [
    W.tfim_small(),
    W.ChainJob("xxz", 8, 8, 8, 4, J=1.0, delta=0.7),
    W.ChainJob("rfheis", 8, 8, 8, 4, J=1.0, fields=tuple(np.linspace(-2, 2, 8))),
    W.ChainJob("tfim_ladder", 8, 8, 8, 4, J=1.0, h=0.9, j_rung=0.5),
    W.tfim_nnn(n_sites=8, leaf_sites=8, k=8),
])
def test_product_terms_match_oracle_hamiltonian_bitwise(job):
    H_prod = _dense(job.n_sites, SM.chain_terms(job))
    H_or = OH.full_hamiltonian(job)
    assert np.array_equal(H_prod, H_or)


def test_block_terms_shift_sites():
    job = W.xxz_chain64()
    t = SM.block_terms(job, 8, 16)
    assert all(0 <= s < 8 for _, ops in t for s, _ in ops)
    assert len(t) == 7 * 3


def test_workloads_deterministic():
    a = W.rfheis_batch(8)
    b = W.rfheis_batch(8)
    assert a == b
    assert all(len(j.fields) == 32 and j.k in (32, 48, 64, 96) for j in a)
    s1 = W.serving_stream(50)
    s2 = W.serving_stream(50)
    assert s1 == s2
    ts = [t for t, _ in s1]
    assert all(t2 > t1 for t1, t2 in zip(ts, ts[1:]))
    assert all(j.n_sites in (16, 32, 64, 128) and 4 <= j.q <= 8 for _, j in s1)


@pytest.mark.parametrize("job,spec", [
    (W.tfim_ladder96(), None),
    (W.ChainJob("xxz", 18, 1, 8, 4, J=1.0, delta=0.8), ((0, 6), ((6, 9), ((9, 12), (12, 18))))),
    (W.ChainJob("tfim_nnn", 16, 1, 8, 4, J=1.0, h=0.7, j2=0.25), (((0, 3), (3, 9)), (9, 16))),
    (W.rfheis_batch(1)[0], (((0, 8), (8, 12)), ((12, 14), (14, 32)))),
])
def test_product_tree_nodes_match_oracle_tree_nodes(job, spec):
    """The product's module-tree builder (spin_models) and the oracle's (oracle.recursion)
    give the same nodes: children, sites, operators and coefficients, in the same order."""
    from oracle import recursion as OR

    if spec is None:
        spec = SM.chain_spec(job.n_sites, job.leaf_sites)
        assert spec == OR.chain_spec(job.n_sites, job.leaf_sites)
    a, b = SM.tree_from_spec(job, spec), OR.tree_from_spec(job, spec)
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x[0] == y[0]
        if x[0] == "leaf":
            assert x[1] == y[1] and x[3] == y[3]
            assert [(c, tuple(ops)) for c, ops in x[2]] == [(c, tuple(ops)) for c, ops in y[2]]
        else:
            assert x[1:3] == y[1:3] and x[4] == y[4]
            assert [tuple(t) for t in x[3]] == [tuple(t) for t in y[3]]


def test_serving_admission_under_sanitizers(tmp_path):
    """The serving admission policy (host code, no GPU) built with the address and
    undefined-behaviour sanitizers and driven through a seeded random stream of
    submissions and completions, checking its invariants after every pass."""
    import shutil
    import subprocess

    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "admission_check")
    src = [os.path.join(ROOT, "tests", "host", "admission_check.cpp"),
           os.path.join(ROOT, "paper_2609_02394_amd", "csrc", "host_util.cpp")]
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                        *src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "admission_check ok" in r.stdout


def test_arena_from_four_threads_under_thread_sanitizer(tmp_path):
    """The arena and the host trace table, which the solver's lanes share, driven from
    four host threads at once under the thread sanitizer (host code, no GPU)."""
    import shutil
    import subprocess

    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "arena_threads_check")
    src = [os.path.join(ROOT, "tests", "host", "arena_threads_check.cpp"),
           os.path.join(ROOT, "paper_2609_02394_amd", "csrc", "host_util.cpp")]
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                        "-I", os.path.join(ROOT, "include"), *src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", RMC_TRACE_HOST="1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "arena_threads_check ok" in r.stdout and "ThreadSanitizer" not in r.stderr


def test_arena_allocator_under_sanitizers(tmp_path):
    """The device-arena sub-allocator (host code, no GPU) built with the address and
    undefined-behaviour sanitizers and driven through a seeded random sequence of
    allocations and releases against a model of the live blocks."""
    import shutil
    import subprocess

    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "arena_check")
    src = [os.path.join(ROOT, "tests", "host", "arena_check.cpp"),
           os.path.join(ROOT, "paper_2609_02394_amd", "csrc", "host_util.cpp")]
    r = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                        *src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "arena_check ok" in r.stdout
