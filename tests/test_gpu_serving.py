"""Serving: many simulations in shared launches (lb_group_*) and the
continuous-batching server.  A member's result must be bit-identical to the
same simulation run alone, whatever else shares its launches and whenever it
joins."""
import sys

import numpy as np
import pytest

import oracle
import paper_1505_03271_amd as lb
import workloads
from paper_1505_03271_amd.serve import Server

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rb_case(n_x, n_y, Ra, Pr, seed, stretch=2.0):
    P = workloads.rb_params(Ra, Pr, n_x, n_y, aspect=n_x / n_y, stretch=stretch)
    return P, workloads.rb_fields(n_x, P["yf"], P["dT"], P["T0"], P["beta_g"], seed_index=seed)


def _rb_oracle(n_x, n_y, Ra, Pr, seed, steps, stretch=2.0):
    """The same Rayleigh-Benard case stepped by the FP64 oracle."""
    P, fields = _rb_case(n_x, n_y, Ra, Pr, seed, stretch)
    c = oracle.Case(n_x, n_y, scheme="heun", wall_y=True, thermal=True, dt=P["dt"], tau=P["tau"], tau_g=P["tau_g"],
                    beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"], T_top=P["T_top"], xf=P["xf"], yf=P["yf"])
    c.init(*fields)
    c.step(steps)
    return c


def _rb_sim(n_x, n_y, Ra, Pr, storage, seed, stretch=2.0):
    P, (rho, ux, uy, T) = _rb_case(n_x, n_y, Ra, Pr, seed, stretch)
    sim = lb.Sim(n_x, n_y, scheme="heun", storage=storage, thermal=True, wall_y=True, dt=P["dt"], tau=P["tau"],
                 tau_g=P["tau_g"], beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"], T_top=P["T_top"],
                 stream=lb.current_stream())
    sim.set_grid(P["xf"], P["yf"])
    sim.init(rho, ux, uy, T)
    return sim


CASES = [(300, 77, 1e7, 1.0, 31), (128, 128, 1e6, 0.7, 45), (200, 150, 1e8, 7.0, 60), (97, 64, 3e6, 1.0, 0)]


@pytest.mark.parametrize("storage,chunk", [("bf16", 0), ("bf16s", 0), ("f32", 0), ("f64", 0), ("bf16s", 24),
                                           ("f64", 8)])
def test_group_members_match_alone_bit_exact(storage, chunk):
    """chunk 0: rows per item chosen by the group at each membership change;
    otherwise fixed."""
    say(f"group vs alone {storage} chunk {chunk}")
    alone = []
    for k, (nx, ny, Ra, Pr, steps) in enumerate(CASES):
        s = _rb_sim(nx, ny, Ra, Pr, storage, 100 + k)
        s.step(steps)
        alone.append(s.get_state())
        s.close()
    sims = [_rb_sim(nx, ny, Ra, Pr, storage, 100 + k) for k, (nx, ny, Ra, Pr, _) in enumerate(CASES)]
    g = lb.Group(8, lb.current_stream())
    g.set_chunk(chunk)
    slots = {}
    for k in (0, 1, 3):
        slots[k] = g.add(sims[k], CASES[k][4])
    g.step(7)
    slots[2] = g.add(sims[2], CASES[2][4])   # joins later: continuous batching
    for _ in range(20):
        g.step(7)
    left = g.remaining()
    assert all(left[slots[k]] == 0 for k in slots)
    for k in range(len(CASES)):
        assert np.array_equal(sims[k].get_state(), alone[k]), f"member {k}"
    if storage == "f64":
        # the group's result is the method's: each FP64 member equals the
        # oracle's run of its case (eq:semi-heun) to 1e-12
        for k, (nx, ny, Ra, Pr, steps) in enumerate(CASES):
            ref = _rb_oracle(nx, ny, Ra, Pr, 100 + k, steps)
            f, gg = sims[k].populations()
            err = max(np.abs(f - ref.f).max() / np.abs(ref.f).max(), np.abs(gg - ref.g).max() / np.abs(ref.g).max())
            say(f"  member {k} ({nx}x{ny}, {steps} steps) vs oracle: {err:.2e}")
            assert err < 1e-12, f"member {k}"
    for k in slots:
        g.remove(slots[k])
    assert g.remaining() == [0] * 8
    g.close()


def test_group_with_a_member_on_separate_launches():
    """A member that does not take fused steps (lb_set_fv_fused(sim, 0))
    makes the group run separate predictor and corrector launches for all
    its members; every member then equals its solo run in that launch shape
    bit for bit, also split 16-bit members, whose default solo steps are
    fused."""
    storage = "bf16s"
    say("group on separate launches")
    cases = CASES[:3]
    alone = []
    for k, (nx, ny, Ra, Pr, steps) in enumerate(cases):
        s = _rb_sim(nx, ny, Ra, Pr, storage, 400 + k)
        s.set_fv_fused(0)
        s.step(steps)
        alone.append(s.get_state())
        s.close()
    sims = [_rb_sim(nx, ny, Ra, Pr, storage, 400 + k) for k, (nx, ny, Ra, Pr, _) in enumerate(cases)]
    sims[1].set_fv_fused(0)
    g = lb.Group(4, lb.current_stream())
    slots = [g.add(sims[k], cases[k][4]) for k in range(len(cases))]
    g.step(max(c[4] for c in cases))
    assert all(n == 0 for n in g.remaining())
    for k in range(len(cases)):
        assert np.array_equal(sims[k].get_state(), alone[k]), f"member {k}"
    for sl in slots:
        g.remove(sl)
    g.close()
    for sim in sims:
        sim.close()


def test_group_membership_rules():
    say("group rules")
    g = lb.Group(2, lb.current_stream())
    a = _rb_sim(64, 64, 1e6, 1.0, "bf16", 1)
    b = _rb_sim(64, 64, 1e6, 1.0, "f32", 2)
    st = lb.Sim(64, 64, scheme="st", storage="bf16", thermal=True, wall_y=True, tau=0.5, tau_g=0.5,
                stream=lb.current_stream())
    st.set_grid(workloads.faces_uniform(64, 64), workloads.faces_uniform(64, 64))
    st.init(np.ones((64, 64)), np.zeros((64, 64)), np.zeros((64, 64)), np.zeros((64, 64)))
    with pytest.raises(lb.LBError) as e:
        g.add(st, 10)
    assert e.value.code == 1
    s0 = g.add(a, 5)
    with pytest.raises(lb.LBError) as e:
        g.add(b, 5)          # different storage format
    assert e.value.code == 1
    with pytest.raises(lb.LBError):
        g.add(a, 5)          # already a member
    c = _rb_sim(64, 64, 1e6, 1.0, "bf16", 3)
    d = _rb_sim(64, 64, 1e6, 1.0, "bf16", 4)
    g.add(c, 0)              # zero steps: never changes
    before = c.get_state()
    with pytest.raises(lb.LBError) as e:
        g.add(d, 5)
    assert e.value.code == 2  # slots full
    g.step(10)
    assert g.remaining()[s0] == 0
    assert np.array_equal(c.get_state(), before)
    g.close()


def test_group_member_changes_only_through_its_group():
    """While in a group a member is neither stepped, re-initialised,
    re-gridded nor re-tuned alone (LB_ESTATE) and joins no second group;
    destroying a member takes it out of its group, whose later launches run
    the other members as before and give its slot to a new member."""
    say("group member guards")
    g, g2 = lb.Group(2, lb.current_stream()), lb.Group(1, lb.current_stream())
    a = _rb_sim(64, 48, 1e6, 1.0, "bf16s", 5)
    b = _rb_sim(80, 64, 1e6, 1.0, "bf16s", 6)
    ref = _rb_sim(80, 64, 1e6, 1.0, "bf16s", 6)
    sa = g.add(a, 20)
    g.add(b, 20)
    P = workloads.rb_params(1e6, 1.0, 64, 48, aspect=64 / 48, stretch=2.0)
    rho, ux, uy, T = workloads.rb_fields(64, P["yf"], P["dT"], P["T0"], P["beta_g"], seed_index=5)
    state = a.get_state()
    calls = [lambda: a.step(1), lambda: a.init(rho, ux, uy, T), lambda: a.set_grid(P["xf"], P["yf"]),
             lambda: a.set_state(state), lambda: a.rebase(), lambda: a.set_fv_lanes(0),
             lambda: a.set_fv_chunk(8), lambda: a.set_rebase(5), lambda: a.set_fv_fused(1), lambda: g2.add(a, 5)]
    for call in calls:
        with pytest.raises(lb.LBError) as e:
            call()
        assert e.value.code == 4
    g.step(10)
    assert g.remaining()[sa] == 10
    a.close()                          # leaves the group first
    assert g.remaining()[sa] == 0
    g.step(10)
    assert g.remaining() == [0, 0]
    ref.step(20)
    assert np.array_equal(b.get_state(), ref.get_state())
    c = _rb_sim(64, 48, 1e6, 1.0, "bf16s", 7)
    assert g.add(c, 5) == sa
    g.step(5)
    assert g.remaining()[sa] == 0
    g.remove(sa)
    c.step(1)                          # alone again
    g.close()
    g2.close()


@pytest.mark.parametrize("policy,min_cells", [("all", 0), ("srpt", 1), ("srpt", 30000)])
def test_server_serves_a_trace_and_results_equal_alone(policy, min_cells):
    """Every request's Nusselt numbers equal those of the same simulation run
    alone, under either policy; with "srpt" and a small min_cells requests
    are preempted (leave the group) and resume later."""
    say(f"server small trace {policy} {min_cells}")
    trace = workloads.serving_trace(n_requests=8, rate=50.0, side=(64, 160), ra=(1e6, 1e8), steps=(40, 160))
    server = Server(storage="bf16", hbm_budget=2e8, max_sims=4, graph_steps=25, policy=policy, min_cells=min_cells)
    stats = server.run(trace)
    server.close()
    assert stats["n_requests"] == 8
    assert stats["p50_s"] > 0 and stats["p99_s"] >= stats["p50_s"]
    by_id = {r["id"]: r for r in stats["requests"]}
    for req in trace:
        solo = Server(storage="bf16", max_sims=1)
        sim = solo._make(req)
        sim.step(req["steps"])
        nu = sim.nusselt()
        sim.close()
        solo.close()
        assert by_id[req["id"]]["nu"] == nu, req["id"]


def test_server_preempts_a_long_request_and_it_resumes_exactly():
    """"srpt" with min_cells 1 runs only the request with the least remaining
    work: a short request that arrives while a long one runs takes its place,
    and the long one resumes afterwards.  Both end with the Nusselt numbers
    of the same simulations run alone."""
    say("server preemption")
    trace = [dict(id=0, arrival=0.0, n=160, Ra=1e7, Pr=1.0, steps=20000),
             dict(id=1, arrival=0.05, n=64, Ra=1e6, Pr=0.7, steps=60)]
    server = Server(storage="bf16s", hbm_budget=2e8, max_sims=4, graph_steps=25, policy="srpt", min_cells=1)
    stats = server.run(trace)
    server.close()
    assert stats["n_requests"] == 2 and stats["preemptions"] >= 1
    by_id = {r["id"]: r for r in stats["requests"]}
    assert by_id[1]["finished"] < by_id[0]["finished"]
    for req in trace:
        solo = Server(storage="bf16s", max_sims=1)
        sim = solo._make(req)
        sim.step(req["steps"])
        nu = sim.nusselt()
        sim.close()
        solo.close()
        assert by_id[req["id"]]["nu"] == nu, req["id"]


def test_server_rejects_a_request_larger_than_the_budget():
    """A request whose memory exceeds the whole HBM budget is rejected and
    listed; every other request is still served."""
    say("server rejects oversize request")
    trace = workloads.serving_trace(n_requests=4, rate=50.0, side=(64, 96), ra=(1e6, 1e7), steps=(20, 40))
    big = dict(trace[1], id=99, n=2048)
    server = Server(storage="bf16", hbm_budget=2e8, max_sims=4, graph_steps=20)
    stats = server.run(trace + [big])
    server.close()
    assert [r["id"] for r in stats["rejected"]] == [99]
    assert sorted(r["id"] for r in stats["requests"]) == sorted(r["id"] for r in trace)


def test_server_lists_a_blown_up_request_as_failed():
    """A request whose time step is far beyond the scheme's stability limit
    (four times the smallest cell) blows up in the group: the kernels raise
    its non-finite flag, the group stops stepping it, and the server lists
    it as failed, with no Nusselt number and out of the latency and
    throughput figures; the other requests are served as usual."""
    say("server lists a blown-up request as failed")
    trace = workloads.serving_trace(n_requests=3, rate=50.0, side=(64, 96), ra=(1e6, 1e7), steps=(40, 80))
    bad = dict(trace[1], id=77, n=64, steps=1500, cfl=4.0)
    server = Server(storage="bf16s", hbm_budget=2e8, max_sims=4, graph_steps=50, policy="all")
    stats = server.run(trace + [bad])
    server.close()
    assert [r["id"] for r in stats["failed"]] == [77]
    assert sorted(r["id"] for r in stats["requests"]) == sorted(r["id"] for r in trace)
    assert all(np.all(np.isfinite(r["nu"])) for r in stats["requests"])


@pytest.mark.parametrize("storage", ["bf16s", "f32", "f16s"])
def test_group_members_renew_their_references_as_alone(storage):
    """Members with a rebase interval (lb_set_rebase) renew their thermal
    references inside the group's captured steps, on the same schedule as
    alone: the state after all steps equals the solo run's bit for bit, also
    for a member that leaves mid-way (its count since the last renewal goes
    with it) and finishes alone, and for members without renewal."""
    say(f"group rebase {storage}")
    cases = [(300, 77, 1e7, 1.0, 57, 10), (128, 128, 1e6, 0.7, 45, 7), (97, 64, 3e6, 1.0, 33, 0),
             (200, 150, 1e8, 7.0, 40, 3)]
    alone = []
    for k, (nx, ny, Ra, Pr, steps, every) in enumerate(cases):
        s = _rb_sim(nx, ny, Ra, Pr, storage, 300 + k)
        s.set_rebase(every)   # 0: none
        s.step(steps)
        alone.append(s.get_state())
        s.close()
    sims = []
    for k, (nx, ny, Ra, Pr, steps, every) in enumerate(cases):
        s = _rb_sim(nx, ny, Ra, Pr, storage, 300 + k)
        s.set_rebase(every)   # 0: none
        sims.append(s)
    g = lb.Group(4, lb.current_stream())
    slots = {k: g.add(sims[k], cases[k][4]) for k in (0, 1, 2)}
    g.step(6)
    slots[3] = g.add(sims[3], cases[3][4])
    g.step(11)
    left1 = g.remaining()[slots[1]]
    g.remove(slots[1])                 # leaves with 4 steps since its last renewal ...
    sims[1].step(int(left1))           # ... and finishes alone
    for _ in range(10):
        g.step(6)
    left = g.remaining()
    assert all(left[slots[k]] == 0 for k in (0, 2, 3))
    for k in range(len(cases)):
        assert np.array_equal(sims[k].get_state(), alone[k]), f"member {k}"
    g.close()
    for s in sims:
        s.close()
