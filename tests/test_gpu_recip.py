"""The reciprocal the setup and raster use for 1/w and 1/A (hardware
reciprocal plus one fused Newton step) against the IEEE division, for every
float it serves: 2^-126 <= x < 2^126, about 2.1e9 values.  The snapped
vertices, weights and depths the parity tests compare bit for bit rest on
this being the correctly rounded quotient; the oracle divides."""
import pytest

from tests.gpu_common import gpu_ctx, note

pytestmark = pytest.mark.gpu


def test_reciprocal_is_the_ieee_quotient():
    import paper_1904_01201_amd as P
    note("reciprocal: exhaustive over [2^-126, 2^126)")
    ctx = gpu_ctx()
    try:
        assert ctx.selfcheck_reciprocal() == 0
        assert ctx.selfcheck_reciprocal(0x3F800000, 0x40000000) == 0    # [1, 2)
        with pytest.raises(P.HabError) as e:
            ctx.selfcheck_reciprocal(0x40000000, 0x3F800000)
        assert e.value.status == P.HAB_ERR_INVALID_ARG
        with pytest.raises(P.HabError):
            ctx.selfcheck_reciprocal(0, 0x80000000)                    # negative floats
    finally:
        ctx.close()
