"""The permutation entry point that allocates nothing (tnc_permute_noalloc),
against the allocating one (tnc_permute) and numpy.transpose: bit-exact, on
two tiled calls in a row (the second smaller, so it runs on the tables the
first one left behind, overwritten in part), a plain-gather call, and the
first shape again.  On the host: tables above the fixed 1 MiB area are
refused before any device work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2606_01852_amd import tnc  # noqa: E402


def test_tables_above_the_fixed_area_are_refused():
    ctx = tnc.Context(-1)
    dummy = 1 << 20   # never dereferenced: refused before any device work
    # (2^17, 64, 64) with the inner 64 x 64 transposed: one tile per outer
    # index, 2^17 outer offsets of 16 bytes = 2 MiB of tables
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_permute_noalloc(ctx.handle, dummy, dummy, (1 << 17, 64, 64), (0, 2, 1))
    assert e.value.status == tnc.E_NOMEM
    with pytest.raises(tnc.TncError) as e:   # within the area: refused only for want of a device
        tnc.tnc_permute_noalloc(ctx.handle, dummy, dummy, (64, 128, 96), (2, 0, 1))
    assert e.value.status == tnc.E_UNSUPPORTED
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_permute_noalloc(ctx.handle, dummy, dummy, (4, 4), (1, 1))
    assert e.value.status == tnc.E_ARG


@pytest.mark.gpu
def test_noalloc_permute_matches_the_allocating_one():
    assert torch.cuda.is_available()
    ctx = tnc.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    cases = [("first, tiled", (64, 128, 96), (2, 0, 1)),
             ("second, smaller, tiled", (2,) * 14, (3, 12, 0, 7, 1, 13, 9, 2, 11, 5, 4, 10, 8, 6)),
             ("plain gather", (3, 4, 5), (2, 0, 1)),
             ("first again", (64, 128, 96), (2, 0, 1))]
    rng = np.random.Generator(np.random.PCG64(2024))
    for name, ext, perm in cases:
        print(f"noalloc permute: {name}, extents {ext}, perm {perm}", flush=True)
        x = (rng.standard_normal(ext + (2,), dtype=np.float32)).view(np.complex64).reshape(ext)
        xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
        y0 = torch.full((x.size,), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
        y1 = torch.full((x.size,), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
        tnc.tnc_permute(ctx.handle, xd.data_ptr(), y0.data_ptr(), ext, perm)
        tnc.tnc_permute_noalloc(ctx.handle, xd.data_ptr(), y1.data_ptr(), ext, perm)
        torch.cuda.synchronize()
        ref = np.ascontiguousarray(np.transpose(x, perm)).reshape(-1)
        got0, got1 = y0.cpu().numpy(), y1.cpu().numpy()
        assert np.array_equal(got1.view(np.uint64), got0.view(np.uint64)), name
        assert np.array_equal(got1.view(np.uint64), ref.view(np.uint64)), name
    ctx.close()
