"""Document front-end (cobs_docset_*): FASTA, multi-FASTA, FASTQ and text
files become documents whose strings are the reads (no q-gram across two
reads) or, for text, the whole file.  Host only: runs without a GPU."""
import numpy as np
import pytest

import paper_1905_09624_amd as cobs

try:
    cobs.lib()
except Exception as e:   # the library must be built for these tests
    pytest.skip(f"libcobs.so not available: {e}", allow_module_level=True)


def strings(ds):
    data, so, dstr = ds.arrays()
    docs = []
    for d in range(len(dstr) - 1):
        docs.append([data[int(so[s]):int(so[s + 1])].tobytes()
                     for s in range(int(dstr[d]), int(dstr[d + 1]))])
    return docs


def wrap(seq, width):
    return b"\n".join(seq[i:i + width] for i in range(0, len(seq), width)) if seq else b""


def test_fasta_records_are_strings_of_one_document(tmp_path):
    rng = np.random.default_rng(1)
    seqs = [rng.choice(np.frombuffer(b"ACGTN", np.uint8), int(n)).tobytes()
            for n in rng.integers(0, 300, 6)]
    text = b";comment line\n" + b"".join(
        b">read%d some description\r\n" % i + wrap(s, 60).replace(b"\n", b"\r\n" if i % 2 else b"\n")
        + b"\n" for i, s in enumerate(seqs))
    p = tmp_path / "doc.fa"
    p.write_bytes(text)
    ds = cobs.DocSet().add_file(str(p), cobs.FASTA).add_buffer(text, cobs.FASTA)
    assert strings(ds) == [seqs, seqs]
    # per-record documents
    assert strings(cobs.DocSet().add_buffer(text, cobs.MULTI_FASTA)) == [[s] for s in seqs]
    # a sequence without a header is one record; whitespace is dropped
    assert strings(cobs.DocSet().add_buffer(b"AC GT\nTT\n", cobs.FASTA)) == [[b"ACGTTT"]]
    assert strings(cobs.DocSet().add_buffer(b"", cobs.FASTA)) == [[]]


def test_fastq_reads(tmp_path):
    reads = [b"ACGTACGT", b"", b"TTTTGGGGCCCCAAAA"]
    text = b"".join(b"@r%d\n%s\n+\n%s\n" % (i, r, b"I" * len(r)) for i, r in enumerate(reads))
    assert strings(cobs.DocSet().add_buffer(text + b"\n", cobs.FASTQ)) == [reads]
    ds = cobs.DocSet()
    for bad in (text[:-3], text.replace(b"+\n", b"-\n", 1), text[:-1] + b"II\n"):
        with pytest.raises(cobs.CobsError) as e:
            ds.add_buffer(bad, cobs.FASTQ)
        assert e.value.status == cobs.EINVAL
    assert strings(ds) == []          # nothing of a refused file is kept
    ds.add_buffer(text, cobs.FASTQ)
    assert strings(ds) == [reads]


def test_text_is_one_continuous_string(tmp_path):
    body = bytes(range(256)) * 3 + b"\n\r\n last line"
    p = tmp_path / "doc.txt"
    p.write_bytes(body)
    assert strings(cobs.DocSet().add_file(str(p), cobs.TEXT)) == [[body]]
    with pytest.raises(cobs.CobsError):
        cobs.DocSet().add_file(str(tmp_path / "missing.txt"), cobs.TEXT)
    with pytest.raises(cobs.CobsError):
        cobs.DocSet().add_buffer(b"x", 99)
