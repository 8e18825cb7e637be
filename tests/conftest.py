import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """(sde module, context handle, torch device) on cuda:0."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0903_3852_amd as sde
    ctx = sde.sde_create(0)
    yield sde, ctx, torch.device("cuda:0")
    torch.cuda.synchronize()
    sde.sde_destroy(ctx)


@pytest.fixture(autouse=True)
def _default_options(request):
    """The GPU context is shared by the session: put every option a test may
    set back to its default afterwards."""
    yield
    if "gpu" in request.fixturenames:
        sde, ctx, _ = request.getfixturevalue("gpu")
        for opt, value in [(sde.SDE_OPT_AUTOTUNE, 1), (sde.SDE_OPT_GRAPHS, 1), (sde.SDE_OPT_JJ_PPT, 0),
                           (sde.SDE_OPT_KURA_MF, 0), (sde.SDE_OPT_KURA_JSPLIT, 0), (sde.SDE_OPT_KURA_TILE, 0),
                           (sde.SDE_OPT_KURA_XCD_LOCAL, 1), (sde.SDE_OPT_KURA_MF_OPT, 0),
                           (sde.SDE_OPT_DENSE_LAUNCH, 0), (sde.SDE_OPT_KURA_MF_PAIRED, 0)]:
            sde.sde_set_option(ctx, opt, value)


def rel_err(got, ref):
    """|got - ref| / max(|ref|, 1), elementwise."""
    import numpy as np
    return np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
