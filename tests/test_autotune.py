"""Selection logic of the tile-shape autotuner on synthetic timings (no GPU)."""
import json

from paper_2107_03958_amd import autotune


def _write(tmp_path, variants, results):
    (tmp_path / "variants.json").write_text(json.dumps(dict(base={"WS_ER64": "16", "WS_CB32": "4",
                                                                  "WS_MIN_BLOCK": "64"},
                                                            variants=variants)))
    (tmp_path / "results_2048.json").write_text(json.dumps(dict(n=2048, results=results)))


def _r(name, prec, defines, total, sample=(1.0, 2.0)):
    return dict(name=name, precision=prec, defines=defines, total_us=total, us_per_density=[total, 0, 0],
                sample=list(sample), scale=2.0)


def test_choose_keeps_faster_correct_shapes(tmp_path, capsys):
    variants = [dict(name="base", precision="both", defines={}),
                dict(name="er8", precision="fp64", defines={"WS_ER64": 8}),
                dict(name="cb2", precision="fp32", defines={"WS_CB32": 2}),
                dict(name="cb8", precision="fp32", defines={"WS_CB32": 8}),
                dict(name="mb256", precision="both", defines={"WS_MIN_BLOCK": 256})]
    results = [_r("base", "fp64", {}, 100.0), _r("base", "fp32", {}, 100.0),
               _r("er8", "fp64", {"WS_ER64": 8}, 95.0),                       # 5% faster: kept
               _r("cb2", "fp32", {"WS_CB32": 2}, 99.5),                       # under 1%: dropped
               _r("cb8", "fp32", {"WS_CB32": 8}, 80.0, sample=(1.0, 2.1)),   # wrong result: rejected
               _r("mb256", "fp64", {"WS_MIN_BLOCK": 256}, 90.0),              # faster in FP64 ...
               _r("mb256", "fp32", {"WS_MIN_BLOCK": 256}, 115.0)]             # ... slower in FP32: dropped
    _write(tmp_path, variants, results)
    out = tmp_path / "tuned.hpp"
    autotune.main(["choose", "--dir", str(tmp_path), "--write", "--out", str(out)])
    text = out.read_text()
    assert "#define WS_ER64 8" in text
    assert "#define WS_CB32 4" in text          # unchanged: cb2 too small a gain, cb8 rejected
    assert "#define WS_MIN_BLOCK 64" in text
    assert "rejected cb8" in capsys.readouterr().out


def test_variants_are_coordinate_neighbours():
    vs = autotune.variants()
    assert vs[0]["name"] == "base" and vs[0]["defines"] == {}
    cur = autotune.current()
    for v in vs[1:]:
        assert len(v["defines"]) == 1
        (k, val), = v["defines"].items()
        assert str(val).replace(" ", "") != cur[k]
