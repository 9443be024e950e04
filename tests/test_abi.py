"""CPU checks of the C ABI: the library loads, exports every symbol that
include/ufss.h declares, and its host-only logic (bin selection, argument
validation) matches the oracle bit for bit.  No GPU call is made."""
import os
import re

import numpy as np
import pytest

from oracle import select as S
from paper_2012_04534_amd import ufss
from paper_2012_04534_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ufss_\w+)\s*\(", text, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = ufss.lib()
    names = declared_symbols()
    assert len(names) >= 11
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(ufss.EXPORTED) <= names


@pytest.mark.parametrize("name", ["bscan32", "cscan32", "cscan64"])
def test_select_freqs_bit_identical_to_oracle(name):
    w = W.workload(name)
    g = w["geom"]
    for seed in (w["seed"], 0, 2 ** 64 - 1):
        b, band = ufss.ufss_select_freqs(g, w["m"], w["per_position"], seed)
        o = S.select_freqs(g, w["m"], w["per_position"], seed)
        assert np.array_equal(b, o)
        assert band == {256: 33, 512: 66, 1024: 132}[g["nt"]]


def test_select_freqs_errors():
    g = W.workload("bscan32")["geom"]
    with pytest.raises(ufss.UfssError) as e:
        ufss.ufss_select_freqs(g, 34, False, 1)
    assert e.value.name == "BAND_TOO_SMALL"
    with pytest.raises(ufss.UfssError) as e:
        ufss.ufss_select_freqs(g, 0, False, 1)
    assert e.value.name == "INVALID_ARG"
    bad = dict(g)
    bad["c"] = -1.0
    with pytest.raises(ufss.UfssError) as e:
        ufss.ufss_select_freqs(bad, 4, False, 1)
    assert e.value.name == "INVALID_ARG"
    full, _ = ufss.ufss_select_freqs(g, 33, False, 9)
    assert list(full) == list(range(10, 43))


@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("name,m", [("bscan32", 1), ("bscan32", 10), ("cscan32", 64),
                                    ("cscan64", 128), ("cscan64", 513)])
def test_sample_bins_bit_identical_to_oracle(strategy, name, m):
    w = W.workload(name)
    g = dict(w["geom"])
    if name != "bscan32":
        g.update(nx=6, ny=5)     # per-position draws in Python stay quick
    band = {256: 33, 512: 66, 1024: 132}[g["nt"]]
    if strategy in (S.STRATEGY_RND, S.STRATEGY_RND_F) and m > band:
        with pytest.raises(ufss.UfssError):
            ufss.ufss_sample_bins(g, m, strategy, 5)
        return
    for seed in (w["seed"], 0, 2 ** 64 - 1):
        b, per = ufss.ufss_sample_bins(g, m, strategy, seed)
        o = S.sample_bins(g, m, strategy, seed)
        assert per == (o.ndim == 3)
        assert np.array_equal(b, o), (strategy, name, m, seed)


def test_sample_bins_errors():
    g = W.workload("bscan32")["geom"]
    with pytest.raises(ufss.UfssError) as e:
        ufss.ufss_sample_bins(g, 130, ufss.SAMPLE_NRG, 1)
    assert e.value.name == "BAND_TOO_SMALL"
    with pytest.raises(ufss.UfssError) as e:
        ufss.ufss_sample_bins(g, 4, 5, 1)
    assert e.value.name == "INVALID_ARG"
    full, _ = ufss.ufss_sample_bins(g, 129, ufss.SAMPLE_NRG, 3)
    assert list(full) == list(range(129))


@pytest.mark.parametrize("name", ["bscan32", "cscan32", "cscan64"])
def test_sigma_estimate_matches_oracle(name):
    from oracle import operator as O
    w = W.workload(name)
    g = dict(w["geom"])
    if name == "cscan32":
        g.update(nx=9, ny=7)      # per-position sums in Python stay quick
    bins = S.select_freqs(g, w["m"], w["per_position"], w["seed"])
    got = ufss.ufss_sigma_estimate(g, w["m"], w["per_position"], bins)
    ref = O.sigma_estimate(g, bins)
    assert got["n"] == ref["n"]
    for k in ("fro_sq", "fro_sq_central", "sigma_hat", "sigma_hat_central"):
        assert got[k] == pytest.approx(ref[k], rel=1e-12), k
    with pytest.raises(ufss.UfssError):
        bad = np.array(bins)
        bad.reshape(-1)[1] = bad.reshape(-1)[0]
        ufss.ufss_sigma_estimate(g, w["m"], w["per_position"], bad)


def test_plan_rejects_bad_bins_before_touching_the_gpu():
    g = W.geometry(8, 4, 16, 64)
    with pytest.raises(ufss.UfssError) as e:
        ufss.Plan(g, 3, False, np.array([5, 4, 6]))
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(ufss.UfssError) as e:
        ufss.Plan(g, 2, False, np.array([5, 40]))
    assert e.value.name == "INVALID_ARG"
    bad = dict(g)
    with pytest.raises(ufss.UfssError) as e:
        ufss.Plan(bad, 2, False, np.array([4, 5]), dtype=ufss.BF16, algo=ufss.ALGO_PHASOR)
    assert e.value.name in ("UNSUPPORTED", "INVALID_ARG")


def header_struct_fields(name):
    """Field names of `typedef struct name {...} name;` in include/ufss.h, in order."""
    text = open(os.path.join(ROOT, "include", "ufss.h")).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1]
        fields += [n.strip().lstrip("*").strip() for n in names.split(",")]
    return fields


@pytest.mark.parametrize("cname,pyname", [("ufss_geom", "Geom"), ("ufss_plan_info", "PlanInfo"),
                                           ("ufss_fista_stats", "FistaStats"),
                                           ("ufss_fista_state", "FistaState"),
                                           ("ufss_tiling", "Tiling"),
                                           ("ufss_sigma_est", "SigmaEst"),
                                           ("ufss_crb_point", "CrbPoint")])
def test_binding_structs_match_header(cname, pyname):
    """The ctypes mirrors of the C structs list the same fields in the same order."""
    cls = getattr(ufss, pyname)
    py = [f.rstrip("_") for f, _ in cls._fields_]
    assert py == header_struct_fields(cname)
