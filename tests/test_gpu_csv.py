"""Extraction of Table-1-shaped text rows into record columns: HIP path vs
the oracle's definition of the row shape, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import assert_exact, check_sort, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl
    cvetl.lib()
    oracle.lib()
    return cvetl


BAD = [b'"q1",2021-05-09 00:00:00,38.1,-92.2,65001,10.5,90', b"x2,2021-02-29 00:00:00,38.1,-92.2,65001,10.5,90",
       b"x3,2021-05-09 00:00:00,3.81e1,-92.2,65001,10.5,90", b"x4,2021-05-09 00:00:00, 38.1,-92.2,65001,10.5,90",
       b"x5,2021-05-09 00:00:00,38.1,-92.2,65001,10.5", b"toolongid,2021-05-09 00:00:00,38.1,-92.2,65001,1,9",
       b"", b"x7,2021-05-09 00:00:00,38.1,-92.2,65001,9007199254740993,9",
       b"x8,2021-05-09 00:00:00.1234,38.1,-92.2,65001,1,9"]
GOOD = [b"y1,2021-05-09 03:48:42,37.664087,-92.6546,65536,105.98,33",
        b"y2,2021-05-09 03:49:42.05,37.667707,-92.6490,65536,0,", b"y3,2021-05-09 23:59:59.999,-0,+0.5,1,.25,359.5",
        b"y4,2020-02-29 12:00:00,1.,-.5,65536,7,0"]


def _text(seed, n_journeys, crlf=False, tail_newline=True):
    r = gen.make_c1(seed=seed, n_journeys=n_journeys, median=500.0, shuffled=True)
    hd = gen.headings(np.random.default_rng(seed), r.journey_id)
    body = gen.to_csv(r, hd, header=False).split(b"\n")[:-1]
    rng = np.random.default_rng(seed)
    extra = BAD + GOOD
    pos = np.sort(rng.integers(0, len(body), len(extra)))
    rows = list(body)
    for p, e in sorted(zip(pos.tolist(), extra), reverse=True):
        rows.insert(p, e)
    eol = b"\r\n" if crlf else b"\n"
    text = gen.CSV_HEADER.rstrip(b"\n") + eol + eol.join(rows) + (eol if tail_newline else b"")
    return text, len(rows)


def _dev(text):
    import torch
    return torch.from_numpy(np.frombuffer(text, dtype=np.uint8).copy()).cuda()


@pytest.mark.parametrize("crlf,tail", [(False, True), (True, True), (False, False)])
def test_csv_extract_matches_oracle(cv, crlf, tail):
    text, n = _text(61, 40, crlf, tail)
    print(f"[csv] bytes={len(text)} rows={n} crlf={crlf} tail_newline={tail}", flush=True)
    rec, hd, ok, r = cv.cv_csv_extract(_dev(text))
    (ej, et, ela, elo, esp), ehd, eok = oracle.csv_extract(text)
    assert r["count"] == n == len(eok) and r["n_bad"] == int((eok == 0).sum()) == len(BAD)
    assert_exact("row_ok", host(ok), eok)
    assert_exact("journey_id", host(rec["journey_id"]), ej)
    assert_exact("ts_ms", host(rec["ts_ms"]), et)
    for name, got, exp in (("lat", rec["lat_deg"], ela), ("lon", rec["lon_deg"], elo)):
        assert_exact(name, host(got).view(np.uint64), exp.view(np.uint64))
    assert_exact("speed", host(rec["speed_mps"]).view(np.uint32), esp.view(np.uint32))
    assert_exact("heading", host(hd).view(np.uint32), ehd.view(np.uint32))


def test_csv_then_sort(cv):
    # extracted records feed the sort; the oracle sorts its own extraction
    text, n = _text(62, 60)
    rec, hd, ok, r = cv.cv_csv_extract(_dev(text))
    keep = host(ok).astype(bool)
    good = {k: v[torch_bool(keep)] for k, v in rec.items()}
    perm, srt, _ = cv.cv_sort_records(good)
    cols, _, eok = oracle.csv_extract(text)
    cols = tuple(c[eok.astype(bool)] for c in cols)
    ep = oracle.sort(cols[0], cols[1])
    check_sort(perm, srt, ep, oracle.sorted_records(cols, ep))


def torch_bool(mask):
    import torch
    return torch.from_numpy(mask).cuda()


def test_csv_edges(cv):
    import torch
    empty = torch.zeros(0, dtype=torch.uint8, device="cuda")
    rec, _, _, r = cv.cv_csv_extract(empty)
    assert r["count"] == 0
    rec, _, ok, r = cv.cv_csv_extract(_dev(b"h\n"))
    assert r["count"] == 0
    rec, _, ok, r = cv.cv_csv_extract(_dev(GOOD[0]), has_header=False)
    assert r["count"] == 1 and int(host(ok)[0]) == 1
    text, n = _text(63, 5)
    with pytest.raises(cv.CvError):
        cv.cv_csv_extract(_dev(text), capacity=n - 1)
