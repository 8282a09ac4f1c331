"""Learned reconstructor trained on simulator frames: what it gains over the
linear reconstructor, and the linear reconstructor as its fallback/judge."""
import numpy as np
import pytest

from synth.configs import CFG2, ATMO2, PUSH_PULL_NM, LOOP_GAIN, LOOP_DELAY
from synth.screens import CropBank, frozen_flow_sequence
from synth.kl import kl_modes
from tests.gpu_common import torch_cuda, say

pytestmark = pytest.mark.gpu

_STATE = {}


def _setup():
    if _STATE:
        return _STATE
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.loop import calibrate
    torch = torch_cuda()
    plan = pw.Plan(CFG2, batch_max=16)
    pupil = plan.pupil.astype(np.float64)
    modes = kl_modes(pupil, CFG2.pixel_m, ATMO2.L0_m, 600).astype(np.float32)
    R, _, _ = calibrate(plan, modes, PUSH_PULL_NM)
    bank = CropBank(CFG2, ATMO2.L0_m, n_screens=2, screen_n=2048, seed=77)
    _STATE.update(plan=plan, pupil=pupil, modes=modes, R=R, bank=bank, torch=torch)
    return _STATE


def test_trained_cnn_beats_linear_in_open_loop_strong_turbulence():
    from paper_1607_07624_amd.learned import train_reconstructor, open_loop_errors
    st = _setup()
    net, info = train_reconstructor(st["plan"], st["R"], st["modes"], st["pupil"], st["bank"], n_frames=49152,
                                    seed=1, epochs=4, batch=256, lr=1e-3, log=say)
    say(f"[gpu] cnn training: {info}")
    assert info["loss_history"][-1] < 0.7 * info["loss_history"][0]
    ev = open_loop_errors(st["plan"], net, st["R"], st["modes"], st["pupil"], st["bank"], 1024, seed=999,
                          r0_range=(0.06, 0.1))
    say(f"[gpu] open-loop modal error, r0 in [0.06, 0.1] m: {ev}")
    assert ev["cnn_nm"] < ev["linear_nm"]
    st["net"] = net


def test_linear_judge_takes_over_from_a_broken_network():
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.cnn import CNN
    from paper_1607_07624_amd.loop import ClosedLoop, residual_rms_nm
    st = _setup()
    torch = st["torch"]
    net = CNN(n_sub=CFG2.n_sub, n_out=600, batch_max=4)
    net.set_params(torch.full((net.n_params,), float("nan"), device="cuda"))
    plan1 = pw.Plan(CFG2, batch_max=1)
    modes_dev = torch.from_numpy(st["modes"]).cuda()
    seq = torch.from_numpy(frozen_flow_sequence(CFG2, ATMO2, 60, seed=3)).cuda()
    cl = ClosedLoop(plan1, modes_dev, st["R"], LOOP_GAIN, LOOP_DELAY, net=net)
    res_c, _ = cl.run(seq)
    assert cl.fallback_step == 0
    lin = ClosedLoop(plan1, modes_dev, st["R"], LOOP_GAIN, LOOP_DELAY)
    res_l, _ = lin.run(seq)
    torch.cuda.synchronize()
    assert torch.equal(res_c, res_l)


def test_linear_judge_takes_over_from_a_diverging_network():
    """A network whose output is a large, input-independent command drives the
    integrator away; the optical-gain probe sees the sensor lose track once the
    settling time is over, the linear reconstructor takes over from zero
    commands and closes the loop again."""
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.cnn import CNN, he_init, PARAM_ORDER
    from paper_1607_07624_amd.loop import ClosedLoop, residual_rms_nm
    st = _setup()
    torch = st["torch"]
    net = CNN(n_sub=CFG2.n_sub, n_out=600, batch_max=4)
    p = he_init(net.shapes, 321)
    off = 0
    for k in PARAM_ORDER:
        n = int(np.prod(net.shapes[k]))
        if k in ("fw2", "fb2"):
            p[off:off + n] *= 300.0
        off += n
    net.set_params(torch.from_numpy(p))
    plan1 = pw.Plan(CFG2, batch_max=1)
    modes_dev = torch.from_numpy(st["modes"]).cuda()
    T = 200
    seq = torch.from_numpy(frozen_flow_sequence(CFG2, ATMO2, T, seed=5)).cuda()
    cl = ClosedLoop(plan1, modes_dev, st["R"], LOOP_GAIN, LOOP_DELAY, net=net)
    res_c, _ = cl.run(seq)
    say(f"[gpu] diverging network: fallback at {cl.fallback_step}, judged {cl.judged}")
    assert cl.fallback_step == cl.judge_settle
    assert all(g > 0.0 for _, g in cl.judged[:1])
    lin = ClosedLoop(plan1, modes_dev, st["R"], LOOP_GAIN, LOOP_DELAY)
    res_l, _ = lin.run(seq)
    pc = residual_rms_nm(res_c.cpu().numpy(), st["pupil"])
    pl = residual_rms_nm(res_l.cpu().numpy(), st["pupil"])
    say(f"[gpu] residual at fallback {pc[cl.fallback_step]:.0f} nm; last 50 steps: "
        f"after fallback {np.sqrt(np.mean(pc[-50:] ** 2)):.1f}, linear {np.sqrt(np.mean(pl[-50:] ** 2)):.1f} nm")
    assert pc[cl.fallback_step] > 5.0 * pl[cl.fallback_step]
    assert np.sqrt(np.mean(pc[-50:] ** 2)) < 1.5 * np.sqrt(np.mean(pl[-50:] ** 2))


@pytest.mark.parametrize("case,L", [("diverging", 50), ("diverging", 7), ("broken", 16), ("random", 10)])
def test_learned_loop_graph_replay_equals_eager(case, L):
    """run_graph with the network: windows end at the judge's steps, the judge
    runs between replays; residuals, commands, the judge's record, the
    hand-over step and the final state equal run()'s bit for bit (with a
    hand-over at step 50, at step 0 and none), also when the graph length
    does not divide the judge's period."""
    import paper_1607_07624_amd as pw
    from paper_1607_07624_amd.cnn import CNN, he_init, PARAM_ORDER
    from paper_1607_07624_amd.loop import ClosedLoop
    st = _setup()
    torch = st["torch"]
    say(f"[gpu] learned graph replay: {case} network, steps per graph {L}")
    net = CNN(n_sub=CFG2.n_sub, n_out=600, batch_max=4)
    if case == "broken":
        net.set_params(torch.full((net.n_params,), float("nan"), device="cuda"))
    else:
        p = he_init(net.shapes, 321)
        if case == "diverging":
            off = 0
            for k in PARAM_ORDER:
                n = int(np.prod(net.shapes[k]))
                if k in ("fw2", "fb2"):
                    p[off:off + n] *= 300.0
                off += n
        net.set_params(torch.from_numpy(p))
    plan1 = pw.Plan(CFG2, batch_max=1)
    modes_dev = torch.from_numpy(st["modes"]).cuda()
    T = 83
    seq = torch.from_numpy(frozen_flow_sequence(CFG2, ATMO2, T, seed=5)).cuda()
    a = ClosedLoop(plan1, modes_dev, st["R"], LOOP_GAIN, LOOP_DELAY, net=net)
    res_a, c_a = a.run(seq)
    b = ClosedLoop(plan1, modes_dev, st["R"], LOOP_GAIN, LOOP_DELAY, net=net)
    for rep in range(2):                                  # the second run replays the kept graphs
        res_b, c_b = b.run_graph(seq, steps_per_graph=L)
        torch.cuda.synchronize()
        say(f"[gpu]   run {rep}: hand-over {a.fallback_step} / {b.fallback_step}, judged {len(a.judged)} / "
            f"{len(b.judged)}, graphs {sorted(b._graphs['graphs'])}")
        assert torch.equal(res_a, res_b) and torch.equal(c_a, c_b)
        assert b.fallback_step == a.fallback_step and [t for t, _ in b.judged] == [t for t, _ in a.judged]
        assert np.array_equal([g for _, g in b.judged], [g for _, g in a.judged], equal_nan=True)
        assert b.state["learned"] == a.state["learned"] and b.state["t"] == a.state["t"]
        assert torch.equal(b.state["commands"], a.state["commands"])
    if case == "diverging":
        assert a.fallback_step == a.judge_settle
    if case == "broken":
        assert a.fallback_step == 0
    net.close()
