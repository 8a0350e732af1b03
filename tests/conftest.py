import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    config.addinivalue_line("markers", "oracle_frames(name): needs the whole-frame oracle of a "
                                       "workload set of tests/oracle_frames.py")


def pytest_collection_finish(session):
    """Synthesise the large phantoms and the whole-frame oracle results the
    selected tests need with worker pools, before any GPU test initialises
    the device (pools are never forked after that)."""
    if not any(item.get_closest_marker("gpu") for item in session.items):
        return
    import oracle_frames
    import phantom
    from phantom.prepare import lighter, prepare

    names = ("pwi", "stai_full", "paper_stai", "paper_pwi", "pwi_batch8")
    full = [phantom.get_workload("pwi"), phantom.get_workload("stai_full")]
    sets = sorted({a for item in session.items
                   for m in item.iter_markers("oracle_frames") for a in m.args})
    frames = [w for name in sets for w in oracle_frames.FRAME_SETS[name]()]
    prepare([lighter(phantom.get_workload(n)) for n in names] + full + frames)
    oracle_frames.prepare(frames)


@pytest.fixture(scope="session")
def wf_gpu():
    """The HIP binding on cuda:0; fails loudly when the GPU or library is missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    import paper_1811_01566_amd as wf

    wf.load()  # raises if libwf.so is missing
    return wf
