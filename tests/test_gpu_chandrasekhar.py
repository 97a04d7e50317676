"""The GPU transport against the exact reflection of a semi-infinite,
isotropically scattering medium at normal incidence (Chandrasekhar's
H-function, tests/hfunc.py): a 40-deep slab with an absorbing surface,
HG g = 0, 1e7 packets, FP32 (the specialised slab kind) and FP64.  Bound:
four times 0.5 / sqrt(N) on the shares, which are means of numbers in
[0, 1]."""
import math

import pytest

from hfunc import HFunction
from test_oracle_chandrasekhar import deep_slab, shares

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2012_00963_amd import pdv
    c = pdv.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("omega,max_orders", [(0.5, 60), (0.9, 400)])
def test_gpu_deep_slab_reflection(ctx, precision, omega, max_orders):
    n = 10_000_000
    p = dict(deep_slab(omega, n, max_orders), precision=precision)
    print("case chandrasekhar", omega, precision, flush=True)
    g = ctx.spectrum(p)
    refl, cone = shares(g, n)
    H = HFunction(omega)
    tol = 4 * 0.5 / math.sqrt(n)
    assert abs(refl - H.plane_albedo()) < tol, (refl, H.plane_albedo())
    assert abs(cone - H.cone_share(math.cos(p["cone_half_angle"]))) < tol, (cone, H.cone_share(math.cos(1.0)))
