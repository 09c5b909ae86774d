"""Host parts of bench.py (CPU): the pass model and the one-GPU refusal."""
import json

import bench


def test_pass_model_is_eleven_n2_s():
    # per density at b = 2: rows n^2 s + 2n^2 s, columns 4n^2 s + (n+1)^2 s, rows 2n^2 s + n^2 s
    for n, s in ((64, 8), (2048, 8), (2048, 4)):
        pb = bench.pass_bytes(n, s)
        assert pb == [3 * n * n * s, 4 * n * n * s + (n + 1) ** 2 * s, 3 * n * n * s]
        assert abs(sum(pb) / (11 * n * n * s) - 1) < 3 / n


def test_period3_pass_model():
    n, s = 1024, 8
    pb = bench.pass_bytes(n, s, b=3)
    inter = 3 * n * n * s
    assert pb == [n * n * s + inter, 2 * inter + (3 * n // 2 + 1) ** 2 * s, inter + n * n * s]


def test_ls_bytes_model():
    # delayed reorthogonalisation: step j reads j basis vectors, u_j and w twice and writes v_j, u_{j+1}
    n, s = 256, 8
    vec = 2 * n * n * s
    assert bench.ls_step_bytes(n, s, 0) == 6 * vec and bench.ls_step_bytes(n, s, 10) == 26 * vec
    info = type("I", (), dict(iterations=3, matvecs=5, refinements=0))()
    # one cycle of 3 columns: 4 steps, 5 operator applications (4 in the cycle, 1 true residual)
    expect = 5 * 27 * n * n * s + sum(bench.ls_step_bytes(n, s, j) for j in range(4)) + 3 * vec
    assert bench.ls_solve_bytes(n, info, False) == expect


def test_table_bytes_is_the_column_pass_extra():
    # the moment table is what the column pass reads beyond the intermediate it reads and writes
    for n, s, b in ((64, 8, 2), (2048, 8, 2), (2048, 4, 2), (1024, 8, 3)):
        assert bench.pass_bytes(n, s, b)[1] - 2 * b * n * n * s == bench.table_bytes(n, s, b)


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert "one GPU" in out["error"] and out["n_gpus"] == 2


def test_paper_timing_density():
    # the density of the paper's timing example (Section 3.1): a normalised Gaussian, sigma = 0.05,
    # about the centre of D; its grid sum times h^2 is its mass, 1
    import synth
    n = 256
    u = synth.gaussian_density(n)
    assert abs(u.sum() / n ** 2 - 1.0) < 1e-12
    assert u[n // 2, n // 2] == u.max()
    assert abs(u.max() - 1.0 / (2 * 3.141592653589793 * 0.05 ** 2)) < 1e-9
