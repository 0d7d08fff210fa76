"""CPU checks of the command line: argument parsing only (no GPU work)."""
import pytest

from paper_2601_11621_amd import cli


def test_parser_accepts_the_three_commands():
    p = cli._parser()
    a = p.parse_args(["factor", "100000", "--out", "f.txt"])
    assert a.cmd == "factor" and a.n == 100000 and a.out == "f.txt"
    a = p.parse_args(["rebuild", "f.txt", "--bin", "c.bin", "--byteorder", "big"])
    assert a.cmd == "rebuild" and a.bin == "c.bin" and a.byteorder == "big" and a.txt is None
    a = p.parse_args(["exact", "10000000", "--decimal", "--reps", "3"])
    assert a.cmd == "exact" and a.decimal and a.reps == 3


def test_parser_rejects_bad_arguments():
    p = cli._parser()
    with pytest.raises(SystemExit):
        p.parse_args(["factor", "100"])                 # --out is required
    with pytest.raises(SystemExit):
        p.parse_args(["exact", "10", "--byteorder", "middle"])
    with pytest.raises(SystemExit):
        p.parse_args([])
