"""Host-side parity of the library's codecs (FPX, AFLP; Sec. 4.1) with the
oracle: stored values and code words bit for bit (hm_codec_column), and the
per-format storage choices of the codec policies for whole matrices
(hm_plan_stats, a host dry run of hm_upload).  No GPU needed."""
import numpy as np
import pytest

import paper_2405_03456_amd as hm
from oracle import codecs, quant, stored, trees
from synth import sphere_points


def _columns(seed, n=40):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n):
        m = int(rng.integers(1, 300))
        col = rng.standard_normal(m) * np.exp(rng.uniform(-6, 6, m) * (t % 3))
        col[rng.random(m) < 0.03] = 0.0
        if t % 7 == 0:
            col[:] = 0.0
        out.append(col)
    out.append(np.array([3.0, -0.75, 0.0, 10.0, 0.1]))
    out.append(np.array([1.0, 1.99999]))
    return out


def test_fpx_codes_match_oracle_bitwise():
    for col in _columns(21):
        for name in ("fpx24", "fpx40", "fpx48", "fpx56", "bf16", "f32"):
            code = stored.DT[name]
            got, words, info = hm.codec_column(name, col)
            want = codecs.fpx_stored(col, code)
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), name
            assert info["dtype"] == name and info["bytes"] == codecs.nbytes(code)
            if codecs.is_fpx(code):
                assert [int(w) for w in words] == [codecs.fpx_bits(float(v), code) for v in want], name


def test_aflp_codes_match_oracle_bitwise():
    for col in _columns(22):
        e0 = codecs.aflp_ebits(col[:, None])
        for e in (e0, e0 + 1, 10):
            for B in range(1, 8):
                name = f"aflp{8 * B}"
                if not codecs.aflp_feasible(B, e):
                    with pytest.raises(hm.HMError):
                        hm.codec_column(name, col, ebits=e)
                    continue
                got, words, info = hm.codec_column(name, col, ebits=e)
                s, z, M, k = codecs.aflp_encode_column(col, e, B)
                want = codecs.aflp_decode(s, z, M, k, e, B)
                assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (name, e)
                assert [int(w) for w in words] == [codecs.aflp_code_word(int(a), int(b), int(c), e, B)
                                                  for a, b, c in zip(s, z, M)], (name, e)
                assert info == {"dtype": name, "bytes": B, "ebits": e, "k": k}


@pytest.mark.parametrize("eps", [0.3, 1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-13, 1e-17])
def test_codec_policies_pick_the_oracle_format(eps):
    for col in _columns(23, 20):
        _, _, info = hm.codec_column("fpx", col, eps=eps)
        assert stored.DT[info["dtype"]] == codecs.fpx_code_for_eps(eps)
        got, _, info = hm.codec_column("aflp", col, eps=eps)
        e = codecs.aflp_ebits(col[:, None])
        B = codecs.aflp_direct_width(e, eps)
        if B is None:
            assert info["dtype"] == "f64" and np.array_equal(got, col)
        else:
            assert info["dtype"] == f"aflp{8 * B}" and info["ebits"] == e
            assert np.array_equal(got, codecs.aflp_stored_column(col, e, B))


def test_codec_column_rejects_bad_input():
    with pytest.raises(hm.HMError):
        hm.codec_column("aflp", [1.0, 2.0])                 # a policy needs eps > 0
    with pytest.raises(hm.HMError):
        hm.codec_column("aflp8", [1.0, np.inf])
    with pytest.raises(hm.HMError):
        hm.codec_column("aflp8", [1.0, 2.0], ebits=8)       # 1 byte cannot hold e = 8
    with pytest.raises(hm.HMError):
        hm.codec_column("aflp24", [1.0, 2.0], ebits=8)      # float32 decode needs e <= 7
    hm.codec_column("aflp32", [1.0, 2.0], ebits=8)


def _case(eps):
    from conftest import cached
    from synth import KERNEL_LAPLACE, compress_h, to_h2, to_uh

    def build():
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p)
        h = compress_h(p, KERNEL_LAPLACE, st, eps, method="svd")
        return p, st, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("valr-host", eps), build)


@pytest.mark.slow
@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
@pytest.mark.parametrize("policy", ["aflp", "fpx", "aflp16", "fpx24"])
def test_codec_plan_counts_match_oracle(eps, policy):
    """hm_plan_stats: the stored entries per format under the codec
    policies (and fixed codec widths) equal the oracle's exactly; the
    stored bytes of the AFLP policy are below those of FPX and of the
    hardware VALR ladder for the H format (the paper finds AFLP compresses
    best, Sec. 4.2)."""
    p, st, vals = _case(eps)
    lay = hm.Layout(p)
    for fmt in ("h", "uh", "h2"):
        counts = np.zeros(stored.NCODES, dtype=np.int64)
        stored.stored_values(st, fmt, vals[fmt], dense=policy, diag=policy, factor=policy, eps=eps, counts=counts)
        s = hm.plan_stats(lay, fmt, vals[fmt], eps=eps, dense=policy, diag=policy, factor=policy)
        assert s["entries_per_dtype"] == [int(c) for c in counts[:17]], fmt
        assert sum(s["bytes_per_dtype"]) == s["bytes_dense"] + s["bytes_factors"] + \
            s["bytes_coupling"] + s["bytes_transfer"]
        if policy == "aflp":
            nominal = sum(c * codecs.nbytes(f) for f, c in enumerate(counts[:17]) if c)
            fc = np.zeros(stored.NCODES, dtype=np.int64)
            stored.stored_values(st, fmt, vals[fmt], dense="fpx", diag="fpx", factor="fpx", eps=eps, counts=fc)
            fpx_nominal = sum(c * codecs.nbytes(f) for f, c in enumerate(fc[:17]) if c)
            assert nominal < fpx_nominal < 8 * counts.sum(), fmt
