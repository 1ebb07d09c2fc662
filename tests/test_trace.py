"""roctx ranges (the serving loop's tick markers): they open and close,
nested, on the host with no tracer attached."""
from paper_2202_13007_amd.trace import Range


def test_ranges_nest_without_a_tracer():
    with Range("outer") as a:
        with Range("inner"):
            pass
    assert a.name == b"outer"
