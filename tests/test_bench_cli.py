"""The benchmark's command line, without a GPU: the default argument list
(one GPU, 20 timed steps, 5 warm-up steps) must parse, and the step counts actually run must keep
the timed window exact and its start on a Gram-Schmidt/measurement period."""
import bench


def test_default_argument_list_parses():
    args = bench.make_parser().parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (args.gpus, args.steps, args.warmup) == (1, 20, 5)
    steps, warmup, prof = bench.plan_counts(args.steps, args.warmup, args.profile_steps, 20)
    assert steps == 20          # timed steps are exactly the requested number
    assert warmup == 20         # rounded up to one whole period
    assert prof % 20 == 0 and prof >= args.profile_steps


def test_defaults_and_off_period_counts():
    args = bench.make_parser().parse_args([])
    assert args.gpus == 1 and args.steps == 200 and args.warmup == 20
    assert bench.plan_counts(200, 20, 20, 20) == (200, 20, 20)
    assert bench.plan_counts(7, 0, 1, 20) == (7, 0, 20)
    assert bench.plan_counts(33, 21, 40, 20) == (33, 40, 40)


def test_more_than_one_gpu_is_refused(capsys):
    import pytest
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "8"])
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
