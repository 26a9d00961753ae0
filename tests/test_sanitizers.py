"""Sanitizer builds of the host-side C and C++ code (CPU only).

AddressSanitizer and UndefinedBehaviorSanitizer builds of
  * the C ABI's host helpers (grim_host.cpp: base packing, exact tolerance
    arithmetic), driven by tests/native/host_helpers_check.c;
  * the oracle (oracle/oracle.c), run through the whole pin suite and the
    chunked comparison driver;
  * the seeded generators (grim_synth/synth.c), run through every generator
    the workloads use, multithreaded.
Any report of the sanitizers fails the test (halt on the first error).  The
sanitized libraries are loaded into a child Python process that preloads the
ASan runtime."""
import os
import subprocess
import sys
import textwrap

import pytest

import grim_synth as gs
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_1711_01177_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def asan_env():
    lib = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                         text=True).stdout.strip()
    if not os.path.isabs(lib) or not os.path.exists(lib):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    env = dict(os.environ)
    env["LD_PRELOAD"] = lib
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    env["PYTHONPATH"] = ROOT
    return env


def test_host_helpers_under_sanitizers(tmp_path):
    env = asan_env()
    env.pop("LD_PRELOAD")  # the program links the runtime itself
    objs = [str(tmp_path / "grim_host.o"), str(tmp_path / "check.o")]
    subprocess.check_call(["g++", "-std=c++17", *SAN, f"-I{INCLUDE}", "-c",
                           os.path.join(CSRC, "grim_host.cpp"), "-o", objs[0]])
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", *SAN, f"-I{INCLUDE}",
                           "-c", os.path.join(ROOT, "tests", "native", "host_helpers_check.c"),
                           "-o", objs[1]])
    exe = str(tmp_path / "host_check")
    subprocess.check_call(["g++", *SAN, *objs, "-o", exe, "-lpthread"])
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


CHILD = textwrap.dedent('''
    import sys
    import numpy as np
    import oracle
    import grim_synth as gs
    from tests import oracle_pins

    orc_path, synth_path = sys.argv[1], sys.argv[2]
    orc = oracle.Oracle(orc_path)
    for check in oracle_pins.ALL_CHECKS:
        check(orc)
    print("pins", len(oracle_pins.ALL_CHECKS), flush=True)

    gs.use_library(synth_path)
    ref = gs.reference(7, 120_003, 0.45, 30, 300, 0.85, 0.98, n_threads=5)
    assert np.array_equal(ref, gs.reference(7, 120_003, 0.45, 30, 300, 0.85, 0.98, n_threads=1))
    rd = gs.reads(3, ref, 3000, [100, 150, 250], [500, 1000], n_threads=4)
    k = gs.cand_counts_zipf(4, 3000, 1.2, 4096)
    k2 = gs.cand_counts_uniform(4, 3000, 1, 2048)
    assert k.max() <= 4096 and k2.max() <= 2048
    off = gs.offsets_from_counts(k)
    cb, tp = gs.cand_random(5, off, rd["read_z"], 200, (ref.size + 199) // 200, n_threads=3)
    kidx = gs.kmer_index(ref, 12)
    so, sb = gs.cand_seeded(ref, kidx, rd["codes"], rd["read_off"], rd["read_len"], 200,
                            n_threads=3)
    for name, scale in (("tiny", 0.05), ("mid", 0.0005), ("batched", 0.00003),
                        ("large", 0.00003)):
        w = gs.make_workload(name, scale=scale, n_threads=3)
        oidx = orc.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=3)
        c, p, bad = orc.filter_batch(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                     w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"],
                                     n_threads=3)
        res = orc.filter_compare(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                 w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"], c,
                                 orc.pack_bitmask(p), n_threads=4, chunk_pairs=5000)
        assert res["count_mismatches"] == 0 and res["bit_mismatches"] == 0, res
        sp, sr, sbn = orc.survivors(orc.pack_bitmask(p), c.size, w["cand_off"], w["cand_bin"])
        d = orc.verify(w["ref"], w["B"], w["O"], w["codes"], w["read_off"], w["read_len"],
                       w["read_e"], w["e_den"], sr[:20], sbn[:20])
        sc = orc.seed_candidates(w["ref"], 12, w["codes"][:20000], w["read_off"][:100],
                                 w["read_len"][:100], w["B"], 4096)
        print(name, c.size, int(p.sum()), int(d.sum()), int(sc[0][-1]), flush=True)
    print("child ok", flush=True)
''')


def test_oracle_and_generators_under_sanitizers(tmp_path):
    env = asan_env()
    orc_lib = str(tmp_path / "liboracle_san.so")
    synth_lib = str(tmp_path / "libgrimsynth_san.so")
    oracle.build(oracle._SRC, orc_lib, extra_flags=SAN)
    gs.build(out=synth_lib, extra_flags=SAN)
    r = subprocess.run([sys.executable, "-c", CHILD, orc_lib, synth_lib], capture_output=True,
                       text=True, env=env, timeout=900, cwd=ROOT)
    assert r.returncode == 0, (r.returncode, r.stdout[-3000:], r.stderr[-6000:])
    assert "child ok" in r.stdout


def test_harness_reports_a_planted_overflow(tmp_path):
    """The sanitized child really runs under ASan: a copy of the oracle with a
    write one vector past the end of its buffer is reported (exit code 86)."""
    env = asan_env()
    with open(oracle._SRC) as f:
        text = f.read()
    old = "vec[t >> 3] |= (uint8_t)(1u << (t & 7));"
    assert text.count(old) == 1
    src = tmp_path / "oracle_overflow.c"
    src.write_text(text.replace(old, "vec[(t >> 3) + nbytes] |= (uint8_t)(1u << (t & 7));"))
    lib = str(tmp_path / "liboracle_overflow.so")
    oracle.build(str(src), lib, extra_flags=SAN)
    code = ("import sys, numpy as np, oracle\n"
            "o = oracle.Oracle(sys.argv[1])\n"
            "ref = np.random.default_rng(1).integers(0, 4, 5000).astype(np.uint8)\n"
            "o.build_bin(ref, 200, 50, 5, 3)\n")
    r = subprocess.run([sys.executable, "-c", code, lib], capture_output=True, text=True, env=env,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 86, (r.returncode, r.stderr[-2000:])
    assert "heap-buffer-overflow" in r.stderr
