"""The benchmark's last stdout line: one JSON object of at most 4 KB with the
fields the measurement contract names, built from a detail record of the
largest size a run produces (every iteration's error, long sample text)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _Args:
    steps, warmup, detail = 20, 5, "bench_detail.json"


def _detail():
    it = _Args.steps + _Args.warmup
    roof = dict(bound="alu", achieved=36.617631, peak=39.3216, unit="Tops/s", frac=0.9312345, traffic=2148532224,
                traffic_algorithmic=2147483648, kernel="fine_kernel<1,double,2> (all 64 slices, one launch)",
                fine_ms=226.123456, fine_particle_steps_per_s=4.6412345e11, ops_per_particle_step=79)
    cfg = dict(workload="slow-fast SDE, eps=0.01, P=2^20 FP64 particles, dt=1e-4, T=10 (1e5 steps), 64 slices, "
                        "1024-cell coarse grid, 100 quantile levels, one parareal iteration per step",
               particles=2 ** 20, fine_steps=100000, slices=64, cells=1024, quantile_levels=100, flags=0, seed=0)
    d = dict(metric=bench.METRIC, value=4.5412345678e11, unit="particle-steps/s", steps=_Args.steps,
             warmup=_Args.warmup, ms_per_step=231.0123456, config=cfg, roofline=roof,
             sweep_roofline=dict(floor_ms=211.0123, measured_ms=231.01234, frac=0.91312345, basis="x" * 120),
             hbm_phases={k: dict(bytes=123456789012, ms=2.6712345, achieved_gbs=4312.12345, frac=0.5312345)
                         for k in ("restrict_fine", "match", "restrict_new")},
             quantile_error=dict(at_T=[1.23456789e-3 / (i + 1) for i in range(it)],
                                 max_over_slices=[2.3456789e-3 / (i + 1) for i in range(it)]),
             serial_fine_s=0.33123456, create_s=1.2345678)
    d["adjoint"] = dict(workload="w" * 300, fwd_plus_adjoint_particle_steps_per_s=1.0123456e11,
                        valu_frac=0.8312345, ops_per_particle_step=306,
                        forward_ckpt_s=0.0251234567, observables_s=0.00123456, reverse_s=0.0791234567,
                        plain_forward_s=0.024123456, reverse_over_forward=3.1234567,
                        ratio_to_8_crn_fd_forwards=0.51234567, jacobian=[[1.0] * 4] * 4, observables=[1.0] * 4,
                        ckpt_every_8=dict(checkpoint_bytes=20971520000, forward_ckpt_s=0.0281234567,
                                          reverse_s=0.0491234567, reverse_over_forward=1.7512345,
                                          jacobian_rel_diff_vs_every256=1.234567e-15))
    d["batched"] = dict(workload="w" * 200, fine_particle_steps_per_iteration=185000000000, work_units=123456,
                        tuned_block=256, tuned_particles_per_thread=2, sweep_ms_graph=466.123456,
                        sweep_ms_batched=455.123456, sweep_ms_per_instance=1031.123456,
                        particle_steps_per_s_graph=3.9712345e11, particle_steps_per_s_per_instance=1.79e11,
                        speedup_vs_per_instance=2.2123456, create_s=5.123456, same_quantile_error=True,
                        iterations_compared=4, sweep_floor_ms=371.123456, sweep_floor_frac_graph=0.8212345)
    d["cpu_baseline"] = dict(value=3.41234567e8, unit="particle-steps/s", cores=16, kind="oracle",
                             sample="s" * 330, cpu_model="AMD EPYC 9575F 64-Core Processor", nproc=256,
                             one_thread=dict(value=2.41234567e7, sample="t" * 60))
    return d


def test_summary_line_fits_and_names_the_contract_fields():
    d = _detail()
    line = bench.summary_line(d, _Args, d["config"])
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) <= 4096, len(text)
    back = json.loads(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "adjoint", "batched"):
        assert k in back, k
    assert back["config"]["workload"] and back["dtype"] == "f64"
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in back["roofline"], k
    assert abs(back["roofline"]["frac"] - back["roofline"]["achieved"] / back["roofline"]["peak"]) < 1e-3
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in back["cpu_baseline"], k
    assert back["batched"]["same_quantile_error"] is True
    assert "reverse_over_forward" in back["adjoint"]
