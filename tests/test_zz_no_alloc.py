"""gmres_encode_noalloc (the entry point that allocates nothing) against gmres_encode."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only hosts
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2011_01850_amd import _lib as L  # noqa: E402

SENTINEL = 0x7A5B


def _encode(lib, fn, prec, w, inv_h, cap):
    out = torch.full((cap,), SENTINEL, dtype=torch.int16, device="cuda")
    sc = C.c_double(-1.0)
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    rc = fn(prec, w.numel(), C.c_void_p(w.data_ptr()), inv_h, C.c_void_p(out.data_ptr()), C.byref(sc),
            C.c_void_p(stream))
    return rc, out.cpu().numpy(), sc.value


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
def test_noalloc_encode_matches_encode_on_calls_in_a_row(fmt):
    lib = L.load()
    prec = L.PRECISIONS[fmt]
    g = np.random.default_rng(17)
    # calls in a row, each smaller than the one before: the largest input the
    # static scratch takes, ragged tails, one element, none.  Large values sit
    # in the last tiles of the earlier calls, so a later call that read their
    # stale partial maxima would get a different scale.
    cases = [(2 ** 24, 3.0), (1_000_003, 1e-3), (65_537, 7.0), (1000, 1e12), (257, 0.5), (1, 2.0), (0, 1.0)]
    for n, mag in cases:
        w_h = (g.standard_normal(n) * mag).astype(np.float32)
        if n > 512:
            w_h[-3] = 1e3 * mag  # the largest magnitude in the ragged last tile
        w = torch.as_tensor(w_h, device="cuda")
        h = float(np.linalg.norm(w_h.astype(np.float64))) or 1.0
        cap = n + 300
        rc_r, ref, sc_r = _encode(lib, lib.gmres_encode, prec, w, 1.0 / h, cap)
        rc_n, got, sc_n = _encode(lib, lib.gmres_encode_noalloc, prec, w, 1.0 / h, cap)
        print(f"{fmt} n={n}: scale {sc_n} (gmres_encode {sc_r})", flush=True)
        assert rc_r == L.OK and rc_n == L.OK, (n, rc_r, rc_n)
        assert sc_n == sc_r, n
        assert np.array_equal(got[:n], ref[:n]), n
        assert np.all(got[n:] == SENTINEL), n  # nothing written past the output
    # beyond the static scratch: refused before any device work
    big = C.c_double()
    assert lib.gmres_encode_noalloc(prec, 2 ** 24 + 1, C.c_void_p(16), 1.0, C.c_void_p(16), C.byref(big),
                                    None) == L.EINVAL
