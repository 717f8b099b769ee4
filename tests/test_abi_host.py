"""CPU-side checks: the C ABI library loads and exports every declared entry
point, the input generators behave as specified, the bench refuses more than
one GPU.  No GPU calls."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1905_09624_amd", "libcobs.so")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cobs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cobs_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(LIB):
        from paper_1905_09624_amd import build
        build.build()
    return LIB


def test_library_exports_every_declared_symbol(built_lib):
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(built_lib)
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/cobs.h but not exported"
    out = subprocess.check_output(["nm", "-D", "--defined-only", built_lib]).decode()
    exported = set(re.findall(r" T (cobs_[a-z_0-9]+)", out))
    assert set(names) <= exported


def test_binding_covers_abi(built_lib):
    import paper_1905_09624_amd as cobs
    assert set(declared_functions()) == set(cobs.EXPORTS)
    cobs.lib()


def test_header_is_plain_c(tmp_path):
    # the boundary is a C ABI: the header compiles as strict C99, with no torch
    # or C++ types, and every declared function is callable from C
    src = tmp_path / "use.c"
    calls = "\n".join(f"    (void)&{f};" for f in declared_functions())
    src.write_text('#include "cobs.h"\nint main(void)\n{\n' + calls + "\n    return 0;\n}\n")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o",
                        str(tmp_path / "use.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


C_PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "cobs.h"

int main(void)
{
    const char *fa = ">r1 first read\nACGT\nAC\n>r2\nTTTT\n";
    const char *fq = "@q\nACGTN\n+\nIIIII\n";
    cobs_docset *ds = NULL;
    cobs_docs docs;
    if (cobs_docset_create(&ds) != COBS_OK) return 1;
    if (cobs_docset_add_buffer(ds, (const uint8_t *)fa, strlen(fa), COBS_FORMAT_MULTI_FASTA) != COBS_OK) return 2;
    if (cobs_docset_add_buffer(ds, (const uint8_t *)fq, strlen(fq), COBS_FORMAT_FASTQ) != COBS_OK) return 3;
    if (cobs_docset_add_buffer(ds, (const uint8_t *)"@x\nAC\n", 7, COBS_FORMAT_FASTQ) != COBS_EINVAL) return 4;
    printf("error: %s\n", cobs_last_error());
    if (cobs_docset_view(ds, &docs) != COBS_OK) return 5;
    printf("docs %u strings %llu bytes %llu\n", docs.n_docs,
           (unsigned long long)docs.doc_str[docs.n_docs],
           (unsigned long long)docs.str_off[docs.doc_str[docs.n_docs]]);
    for (uint32_t d = 0; d < docs.n_docs; ++d)
        for (uint64_t i = docs.doc_str[d]; i < docs.doc_str[d + 1]; ++i)
            printf("doc %u: %.*s\n", d, (int)(docs.str_off[i + 1] - docs.str_off[i]),
                   (const char *)docs.bytes + docs.str_off[i]);
    cobs_docset_free(ds);
    if (cobs_set_allocator(NULL) != COBS_OK) return 6;
    return 0;
}
"""


def test_c_program_links_and_calls_the_library(built_lib, tmp_path):
    # a plain C program linked against libcobs.so uses the host-side entry
    # points (document sets from FASTA/FASTQ buffers, errors) without Python
    src = tmp_path / "prog.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "prog"
    libdir = os.path.dirname(built_lib)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(exe), "-L", libdir, "-lcobs",
                        "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    lines = r.stdout.splitlines()
    assert lines[0].startswith("error: ") and "FASTQ" in lines[0]
    assert lines[1] == "docs 3 strings 3 bytes 15"
    assert lines[2:] == ["doc 0: ACGTAC", "doc 1: TTTT", "doc 2: ACGTN"]


def test_allocator_needs_a_free_function(built_lib):
    # host-side argument check of cobs_set_allocator (no device memory touched)
    import paper_1905_09624_amd as cobs
    lonely = cobs.Allocator(cobs._ALLOC_FN(lambda ctx, n: None), cobs._FREE_FN(), None)
    assert cobs.lib().cobs_set_allocator(ctypes.byref(lonely)) == cobs.EINVAL
    assert cobs.lib().cobs_set_allocator(None) == cobs.OK


def test_product_path_fails_loudly_without_the_library():
    # with libcobs.so absent every entry point raises; nothing falls back
    code = ("import numpy as np, paper_1905_09624_amd as c\n"
            "c.LIB_PATH = '/nonexistent/libcobs.so'\n"
            "prm = c.make_params(0, 31, True, 1, 0.3, 0, 1)\n"
            "d = np.frombuffer(b'ACGT' * 20, np.uint8)\n"
            "try:\n"
            "    c.Index.build(prm, d, np.array([0, 80], np.uint64), np.array([0, 1], np.uint64))\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "not built" in r.stdout


def test_library_does_not_link_the_oracle(built_lib):
    out = subprocess.check_output(["nm", "-D", built_lib]).decode()
    assert "orc_" not in out
    deps = subprocess.check_output(["ldd", built_lib]).decode()
    assert "oracle" not in deps


def test_product_sources_do_not_reference_oracle():
    pkg = os.path.join(ROOT, "paper_1905_09624_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dp, f)).read()
                assert "import oracle" not in text and "cobs_oracle" not in text, f


# ---- generator ---------------------------------------------------------------

def test_philox_known_answers():
    # Random123 known-answer vectors for Philox4x32-10
    assert synth.philox([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert synth.philox([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                        [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420,
                                                      0x24126EA1]


def test_doc_lengths_follow_recipes():
    w1 = synth.CONFIGS[1]
    l1 = synth.doc_lengths(w1)
    assert l1.min() >= 10_000 and l1.max() <= 100_000
    assert abs(l1.mean() - 55_000) < 3_000
    w3 = synth.CONFIGS[3].scaled(100)
    l3 = synth.doc_lengths(w3).astype(np.float64) - 30
    med = np.median(l3)
    assert 0.85 * 1e4 < med < 1.15 * 1e4
    assert l3.max() <= 8e4
    sig = np.std(np.log(np.maximum(l3[l3 < 8e4], 1)))
    assert 0.6 < sig < 0.8


def test_docs_are_deterministic_and_uniform():
    w = synth.CONFIGS[1].scaled(100)
    a = synth.dna_docs(w)
    b = synth.dna_docs(w)
    assert np.array_equal(a.bytes, b.bytes)
    counts = np.bincount(a.bytes, minlength=256)
    sd = (0.25 * 0.75 / a.bytes.size) ** 0.5
    assert counts[[ord(c) for c in "ACGT"]].sum() == a.bytes.size
    for c in b"ACGT":
        assert abs(counts[c] / a.bytes.size - 0.25) < 4 * sd
    # random access agrees with the bulk generator
    for d in (0, 3):
        off = int(a.str_off[d])
        for i in (0, 1, 63, 64, 100):
            assert synth.doc_base(w.seed, d, i) == a.bytes[off + i]


def test_planted_queries_copy_their_source():
    w = synth.CONFIGS[2].scaled(100)
    d = synth.dna_docs(w)
    qs = synth.dna_queries(w, n=40)
    planted = [i for i in range(qs.n) if qs.src[i] >= 0]
    assert len(planted) == 20
    total = diff = 0
    for i in planted:
        q = np.frombuffer(qs.get(i), np.uint8)
        doc = d.bytes[int(d.str_off[qs.src[i]]):int(d.str_off[qs.src[i] + 1])].tobytes()
        # find the offset by matching the longest exact prefix
        best = None
        for off in range(len(doc) - len(q) + 1):
            mism = np.count_nonzero(np.frombuffer(doc[off:off + len(q)], np.uint8) != q)
            if best is None or mism < best:
                best = mism
            if mism <= 0.05 * len(q):
                break
        total += len(q)
        diff += best
    assert 0.004 < diff / total < 0.02


def test_text_generator_shapes():
    w = synth.CONFIGS[4].scaled(1000)
    d = synth.text_docs(w)
    lens = np.diff(d.str_off.astype(np.int64))
    assert lens.min() >= 1
    assert np.count_nonzero(d.bytes == 0x20) > 0.05 * d.bytes.size
    qs = synth.text_queries(w, d, n=10)
    assert all(16 <= len(qs.get(i)) <= 4096 for i in range(qs.n))


def test_arrivals_are_poisson():
    t = synth.arrivals(7, 20000, 1000.0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1e-3) < 5e-5
    assert abs(gaps.std() - 1e-3) < 1e-4


def test_bench_reads_traffic_only_for_the_current_kernel(tmp_path, monkeypatch):
    # roofline.traffic comes from the committed counter summary, and only
    # while the kernel source it was taken with is unchanged
    sys.path.insert(0, ROOT)
    import bench
    assert bench.committed_traffic("text-50k") is None          # another workload
    t = bench.committed_traffic("compact-100k")
    assert t is None or t > 266_739_329_024                     # at least the rows it must read
    changed = tmp_path / "gather.hip"
    changed.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(changed))
    assert bench.committed_traffic("compact-100k") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_bench_cpu_baseline_on_a_whole_block():
    # the CPU-baseline leg on a small compact plan: a whole block of 1,024
    # documents as sub-indexes at the block's row count, the per-lookup and
    # per-document model, and its check on the half block
    sys.path.insert(0, ROOT)
    import bench
    import oracle
    from dataclasses import replace
    w = replace(synth.CONFIGS[3].scaled(40), B=1024)
    lens = synth.doc_lengths(w).astype(np.int64)
    n_terms = lens - 30           # the exact counts do not matter for the timing
    order = np.lexsort((np.arange(w.n_docs), n_terms))
    qs = synth.dna_queries(w, n=20)
    r = bench.cpu_baseline_block(w, synth, oracle, qs, order, n_terms, 1.5, 2)
    assert r["kind"] == "oracle" and r["cores"] == 2
    assert r["value"] > 0 and r["value_1_thread"] > 0
    assert r["ns_per_lookup"] > 0 and r["ns_per_lookup_document"] > 0
    assert "block 0 of the compact plan" in r["sample"] and "1025 columns" in r["sample"]
