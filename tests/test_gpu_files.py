"""Index files: an index written with cobs_index_save and read back with
cobs_index_load (into device memory, or kept in host memory and streamed) is
the same index: layout, matrix bytes and every query result.  Damaged files
are refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WORKLOADS = {
    "compact": synth.CONFIGS[3].scaled(50),
    "classic": synth.CONFIGS[1].scaled(4),
    "text": synth.CONFIGS[4].scaled(100),
}


@pytest.fixture(scope="module", params=sorted(WORKLOADS))
def built(request):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    w = WORKLOADS[request.param]
    d = synth.docs(w)
    kind = 0 if w.kind == "dna" else 1
    prm = cobs.make_params(kind, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    qs = synth.dna_queries(w, n=30) if w.kind == "dna" else synth.text_queries(w, d, n=30)
    return cobs, w, ix, qs


def _same_index(a, b, qs):
    ia, ib = a.info(), b.info()
    for k in ("n_docs", "n_blocks", "total_bytes", "score_bytes"):
        assert ia[k] == ib[k], k
    for x, y in zip(a.order(), b.order()):
        assert np.array_equal(x, y)
    for blk in range(ia["n_blocks"]):
        assert a.block(blk) == b.block(blk)
    assert np.array_equal(a.read(0, ia["total_bytes"]), b.read(0, ib["total_bytes"]))
    for k, topk in (((1, 2), 0), ((0, 1), 4)):
        for x, y in zip(a.query(qs.bytes, qs.q_off, k=k, topk=topk),
                        b.query(qs.bytes, qs.q_off, k=k, topk=topk)):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]


def test_save_load_roundtrip(built, tmp_path):
    cobs, w, ix, qs = built
    path = str(tmp_path / "index.cobs")
    ix.save(path)
    back = cobs.Index.load(path)
    assert not back.info()["host_resident"]
    _same_index(ix, back, qs)
    # kept in host memory, streamed through a budget of twice the largest block
    info = ix.info()
    big = max(ix.block(b)["rows"] * ix.block(b)["stride"] for b in range(info["n_blocks"]))
    host = cobs.Index.load(path, device_budget_bytes=2 * ((big + 255) // 256 * 256))
    assert host.info()["host_resident"]
    _same_index(ix, host, qs)
    # a loaded index saves to the same bytes
    path2 = str(tmp_path / "again.cobs")
    host.save(path2)
    assert open(path, "rb").read() == open(path2, "rb").read()


def test_damaged_files_are_refused(built, tmp_path):
    cobs, w, ix, qs = built
    path = tmp_path / "index.cobs"
    ix.save(str(path))
    good = path.read_bytes()
    header = 8 + 4 * 6 + 8 + 8 + 4 * 2 + 8 * 3

    def refused(data, name):
        p = tmp_path / name
        p.write_bytes(data)
        with pytest.raises(cobs.CobsError) as e:
            cobs.Index.load(str(p))
        assert e.value.status == cobs.EINVAL

    refused(b"XOBS" + good[4:], "magic.cobs")
    refused(good[:header - 3], "short_header.cobs")
    refused(good[:header + 10], "short_meta.cobs")
    refused(good[:len(good) - 1], "short_matrix.cobs")
    flipped = bytearray(good)
    flipped[header + 1] ^= 0x01                       # the order array
    refused(bytes(flipped), "checksum.cobs")
    with pytest.raises(cobs.CobsError) as e:
        cobs.Index.load(str(tmp_path / "missing.cobs"))
    assert e.value.status == cobs.EINVAL
