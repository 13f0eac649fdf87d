import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


_LIB_CHECK = []


@pytest.fixture(autouse=True)
def _library_built_from_these_sources(request):
    """GPU tests must exercise a library built from the sources in this tree:
    the build embeds a hash of its sources in gc_version()."""
    if request.node.get_closest_marker("gpu") is None:
        return
    if not _LIB_CHECK:
        from paper_2511_22094_amd import build, lib
        want = build.source_hash()
        got = lib().gc_version()
        _LIB_CHECK.append((want in got, want, got))
    ok, want, got = _LIB_CHECK[0]
    assert ok, (f"libgacelle.so ({got}) was not built from these sources (hash {want}): "
                "rebuild with `python -m paper_2511_22094_amd.build`")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
