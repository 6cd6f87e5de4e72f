"""The LDS bandwidth probe (a measurement aid for the bench's roofline) runs
and returns a plausible figure: above 1 TB/s, below 1 PB/s."""
import pytest

pytestmark = pytest.mark.gpu


def test_lds_probe():
    import paper_2208_05795_amd as tsg
    with tsg.Context(0) as ctx:
        bw = ctx.probe_lds()
    print(f"[gpu] LDS read bandwidth {bw / 1e12:.1f} TB/s", flush=True)
    assert 1e12 < bw < 1e15
