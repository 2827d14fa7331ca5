"""The planner (host code of libnnef) without a GPU, through nnef_plan_dry:
which lowering each block gets, the tile geometry, and its invariants."""
import math
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.skipif(
    not os.path.exists(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                    "paper_2602_02759_amd", "libnnef.so")),
    reason="libnnef.so is not built")


def dry(*args, **kw):
    from paper_2602_02759_amd.nnef import nnef_plan_dry
    return [parse(line) for line in nnef_plan_dry(*args, **kw).strip().splitlines()]


def parse(line):
    d = {"op": re.search(r"'([a-zA-Z]+)'", line).group(1), "direct": "': direct " in line}
    if d["direct"]:
        for key in ("P", "Q", "R", "S"):
            d[key] = re.search(rf"\b{key}={{([a-zA-Z]*)}}", line).group(1)
        for key in ("K", "KS", "nP", "nQ", "grid", "chunks", "threads/entry", "rows/wg"):
            d[key] = int(re.search(rf"\b{re.escape(key)}=(\d+)", line).group(1))
        d["contract"] = re.search(r"contract=(\w+)", line).group(1)
        d["permute"] = "permute-back" in line
        return d
    for key in ("P", "Q", "kappa", "qo"):
        d[key] = re.search(rf"\b{key}={{([a-zA-Z]*)}}", line).group(1)
    for key in ("K", "KP", "nP", "nQ", "grid", "chunks", "steps/wave"):
        d[key] = int(re.search(rf"\b{re.escape(key)}=(\d+)", line).group(1))
    d["L"] = re.search(r"\bL=(\w+)", line).group(1)
    d["R"] = re.search(r"\bR=(materialised|product\([a-zA-Z,\[\]]+\))", line).group(1)
    d["qi"] = re.search(r"\bqi=([a-zA-Z-])", line).group(1)
    d["contract"] = re.search(r"contract=(\w+)", line).group(1)
    d["vecq"] = " vecq" in line
    d["chain"] = "chain-back" in line
    d["wave_rows"] = "wave-rows" in line
    return d


def test_cp3_headline_lowering():
    b = dry("ir,jr,kr->ijk", [256, 256, 256], [32], 1.0, 1.0)
    assert [x["op"] for x in b] == ["ir", "jr", "kr"]
    for x, (p, rest) in zip(b, [("i", "jr,kr"), ("j", "ir,kr"), ("k", "ir,jr")]):
        assert x["P"] == p and x["L"] == "direct" and x["R"] == f"product({rest})" and not x["chain"]
        assert (x["K"], x["KP"], x["nP"], x["nQ"]) == (32, 32, 256, 65536)
        assert (x["grid"], x["chunks"], x["steps/wave"]) == (512, 64, 8)
    assert b[0]["vecq"] and b[1]["vecq"] and not b[2]["vecq"]  # k is innermost in Y


def test_manybody_takes_the_direct_lowering():
    """No split of 'ij,jk,ik->ijk' keeps every operand on one side: each block
    sums its entries directly (rows = the operand's own modes), with no
    buffer the size of the data."""
    b = dry("ij,jk,ik->ijk", [96, 96, 96], [], 1.0, 0.0)
    assert all(x["direct"] for x in b)
    assert [(x["P"], x["Q"], x["K"], x["KS"]) for x in b] == [("ij", "k", 1, 1), ("jk", "i", 1, 1),
                                                               ("ik", "j", 1, 1)]
    assert all(x["nP"] * x["nQ"] == 96 ** 3 and x["threads/entry"] == 1 for x in b)


def test_rank_above_64_takes_the_direct_lowering():
    b = dry("ir,jr,kr->ijk", [128, 128, 128], [96], 1.0, 0.0, prec="bf16")
    assert all(x["direct"] and x["K"] == 96 and x["R"] == "r" and x["S"] == "" for x in b)
    assert all(x["threads/entry"] == 8 and x["contract"] == "fp32" for x in b)


def test_direct_lowering_with_other_latents_and_a_permuted_operand():
    # r lives only in the first operand (summed there), which is laid out r-first
    b = dry("rij,jk,ik->ijk", [13, 11, 9], [3], 1.0, 0.0)
    assert all(x["direct"] for x in b)
    assert (b[0]["R"], b[0]["S"], b[0]["permute"]) == ("r", "", True)
    assert (b[1]["R"], b[1]["S"], b[1]["KS"], b[1]["permute"]) == ("", "r", 3, False)


def test_beyond_the_direct_lowering_is_rejected():
    from paper_2602_02759_amd.nnef import NnefError, nnef_plan_dry
    with pytest.raises(NnefError) as e:
        nnef_plan_dry("ir,jr,kr->ijk", [40, 30, 20], [300])
    assert e.value.status == 7 and "direct lowering" in str(e.value)


@pytest.mark.parametrize("model,sizes,ranks", [
    ("ij,jk,ik->ijk", [19, 17, 13], []), ("ir,jr,kr->ijk", [40, 30, 20], [96]),
    ("ia,jb,kc,abc->ijk", [30, 26, 18], [6, 5, 4]), ("ia,jab,kbc,lc->ijkl", [13, 11, 9, 7], [3, 4, 5]),
    ("wr,dr,hr,irk,jrk->wdhij", [27, 7, 24, 10, 10], [10, 6]), ("ij,i->ij", [30, 20], [])])
def test_no_block_materialises_the_reconstruction(model, sizes, ranks):
    """No lowering holds a buffer with one value per data entry: either a
    bilinear split with a non-empty column side, or the direct lowering."""
    for x in dry(model, sizes, ranks, 1.0, 0.0):
        assert x["direct"] or x["Q"] != ""


def test_tucker_lowering_and_precision_per_width():
    b = dry("ia,jb,kc,abc->ijk", [512, 512, 128], [32, 32, 16], 1.0, -1.0, prec="bf16")
    assert [x["L"] for x in b] == ["direct", "direct", "direct", "materialised"]
    assert [x["KP"] for x in b] == [32, 32, 16, 32]
    # BF16 contraction inputs at every width (32x32 tiles at 32, 16x16 tiles at 16)
    assert [x["contract"] for x in b] == ["bf16", "bf16", "bf16", "bf16"]
    assert b[3]["chain"] and b[3]["wave_rows"]          # core: 65,536 rows, 16 column steps
    assert not any(x["wave_rows"] for x in b[:3])


def test_tensor_train_and_icews_lowerings():
    tt = dry("ia,jab,kbc,lc->ijkl", [128, 128, 96, 64], [16, 16, 16], 1.0, 0.0)
    assert all(x["KP"] == 16 for x in tt)
    assert sum(x["chain"] for x in tt) >= 2
    ic = dry("ir,jr,ak,kr,tr->ijat", [249, 249, 20, 228], [32, 8], 1.0, 0.0)
    # no block materialises a row side of one row per (i, a, t): the rows of
    # block ir are (i, a), the columns the product of jr and tr rows
    assert (ic[0]["P"], ic[0]["R"], ic[0]["qi"]) == ("ia", "product(jr,tr)", "t") and ic[0]["vecq"]
    assert (ic[1]["P"], ic[1]["R"]) == ("ja", "product(ir,tr)")
    assert all(x["nP"] <= 4980 for x in ic)
    assert ic[2]["R"] == "product(ir,jr)"


def test_grouped_column_pieces():
    """Column-side operands linked by a latent letter outside kappa form one
    piece, contracted into a small buffer before the pass: in block ir of
    'ir,jr,ak,kr->ija' the columns (j, a) are the product of jr rows and rows
    of [a, r] = sum_k ak kr."""
    b = dry("ir,jr,ak,kr->ija", [64, 48, 40], [16, 4], 1.0, 0.0)
    assert (b[0]["P"], b[0]["Q"], b[0]["R"], b[0]["L"]) == ("i", "ja", "product(jr,[ar])", "direct")
    assert not b[0]["chain"]


def test_latent_only_operand_and_shared_letter():
    b = dry("ir,jr,jkr->ijk", [21, 18, 20], [5], 1.0, 0.0)
    assert len(b) == 3
    b = dry("ia,jb,ab->ij", [30, 20], [4, 3], 1.0, 0.0)
    assert b[2]["op"] == "ab"


def test_low_rank_tucker_and_wits_lowerings():
    # Tucker with a CP-factored core: every block contracts over the core's CP
    # rank r, including the latent-only operands ar, br, cr
    b = dry("ia,jb,kc,ar,br,cr->ijk", [512, 512, 128], [32, 32, 16, 8], 1.0, -1.0)
    assert [x["op"] for x in b] == ["ia", "jb", "kc", "ar", "br", "cr"]
    assert all(x["kappa"] == "r" and x["K"] == 8 and x["KP"] == 16 for x in b)
    assert all(x["chain"] for x in b)
    # the paper's trade-data string: rank-32 CP with a rank-4 time factor
    b = dry("er,ir,gr,tk,kr->eigt", [196, 196, 96, 29], [32, 4], 1.0, -0.5)
    assert [x["op"] for x in b] == ["er", "ir", "gr", "tk", "kr"]
    assert all(x["kappa"] == "r" and x["K"] == 32 for x in b)
    for x in b:
        assert x["nP"] * x["nQ"] == 196 * 196 * 96 * 29


@pytest.mark.parametrize("seed", range(6))
def test_geometry_invariants_on_random_cp(seed):
    """For random CP shapes and ranks: the grid is panels x chunks, the chunks
    cover every column step, and the padded width is the next of 16/32/64."""
    rng = np.random.default_rng(seed)
    dims = [int(v) for v in rng.integers(5, 300, size=3)]
    R = int(rng.choice([3, 8, 16, 24, 32, 40, 64]))
    for x in dry("ir,jr,kr->ijk", dims, [R], 1.0, 0.0):
        assert not x["direct"]
        assert x["KP"] == (16 if R <= 16 else 32 if R <= 32 else 64) and x["K"] == R
        qstep = 16 if x["KP"] == 16 else 32
        rows = 64 if x["KP"] == 16 else (128 if x["wave_rows"] else 32)
        panels = math.ceil(x["nP"] / rows)
        assert x["grid"] == panels * x["chunks"]
        nqi = {"i": dims[0], "j": dims[1], "k": dims[2]}[x["qi"]]
        n_steps = (x["nQ"] // nqi) * math.ceil(nqi / qstep)
        split = 1 if x["wave_rows"] else 4
        assert x["chunks"] * split * x["steps/wave"] >= n_steps
        assert (x["chunks"] - 1) * split * x["steps/wave"] < n_steps


def test_dry_run_reports_the_same_errors():
    from paper_2602_02759_amd.nnef import NnefError, nnef_plan_dry
    with pytest.raises(NnefError) as e:
        nnef_plan_dry("ii,jr->ij", [4, 5], [3])
    assert e.value.status == 1
    with pytest.raises(NnefError) as e:
        nnef_plan_dry("ir,jr->ij", [4, 5], [3], 0.0, 0.5)
    assert e.value.status == 3
    with pytest.raises(NnefError) as e:
        nnef_plan_dry("ir,jr->ij", [4, 5], [3], family="negbin", family_param=-1.0)
    assert e.value.status == 3
    assert dry("ir,jr->ij", [4, 5], [3], family="js")
