"""The persistent batched launch's schedule (mpdet_batched_plan, host only):
every phase of every matrix appears once, in its matrix's own order, with the
dependency counts the kernel waits for; and the queue protocol the kernel
follows (tickets taken in order by whichever workgroup is free, a ticket
starts when its matrix's completed-ticket count reaches the record's `need`)
drains for any number of workgroups, emulated here on the CPU with random
progress, never starting a phase before every earlier phase of its matrix is
complete."""
import os

import numpy as np
import pytest

from paper_1308_1536_amd import binding

WAVES = 4  # waves per workgroup: one unit each per ticket


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmpdet.so is not built (run __graft_entry__.build())")
    return binding.lib()


def expected_phases(n, P, minors):
    """A matrix's phases in order: (kind, k, units), restating the schedule the
    header describes (lane product for P <= 128, P % 4 == 0, with the next
    pivot examined by the finish; the one-wave update otherwise)."""
    lane = P <= 128 and P % 4 == 0
    out = [("init", 0, 1)]
    for k in range(n):
        m = n - k - 1
        if not lane or k == 0:
            out.append(("pivot", k, 2))
        if m <= 0:
            continue
        out.append(("divide", k, m))
        if lane:
            out.append(("prod", k, -(-m // 4) * -(-m // 64)))
            out.append(("finish", k, m * -(-m // 64)))
        else:
            out.append(("updv", k, m * m))
    out.append(("pend", n - 1, 1))
    if minors:
        for s in range(n - 1):
            out.append(("msweep", n - 1 - s, n - 1 - s))
        out.append(("mfinal", 0, n))
    return out


def tickets(kind, units):
    return units if kind in ("init", "prod", "pend") else -(-units // WAVES)


CASES = [([5, 3, 1], 8, True), ([17, 40, 2, 33, 9, 64, 1], 16, True), ([30, 12, 29], 64, False),
         ([7, 20, 3], 6, True), ([11, 4], 130, True), ([1], 64, True)]


@pytest.mark.parametrize("sizes,P,minors", CASES)
def test_plan_lists_every_phase_in_order(lib, sizes, P, minors):
    recs, total = binding.batched_plan(sizes, P, "valu", minors)
    assert total == sum(tickets(binding.PLAN_KINDS[r["kind"]], int(r["units"])) for r in recs)
    for b, n in enumerate(sizes):
        mine = recs[recs["mat"] == b]
        got = [(binding.PLAN_KINDS[r["kind"]], int(r["k"]), int(r["units"])) for r in mine]
        assert got == expected_phases(n, P, minors), f"matrix {b}"
        run = 0
        for r in mine:
            assert r["need"] == run
            run += tickets(binding.PLAN_KINDS[r["kind"]], int(r["units"]))


def test_plan_order_is_step_then_phase_then_size(lib):
    sizes = [9, 30, 14]
    recs, _ = binding.batched_plan(sizes, 8, "valu", True)
    # at elimination step 0 the largest matrix's multipliers come first
    div0 = [int(r["mat"]) for r in recs if binding.PLAN_KINDS[r["kind"]] == "divide" and r["k"] == 0]
    assert div0 == [1, 2, 0]


@pytest.mark.parametrize("workers", [1, 2, 7, 64])
@pytest.mark.parametrize("sizes,P,minors", CASES[:4])
def test_queue_protocol_drains(lib, sizes, P, minors, workers):
    recs, total = binding.batched_plan(sizes, P, "valu", minors)
    # ticket -> (record, matrix, need); record completion bookkeeping
    kinds = [binding.PLAN_KINDS[r["kind"]] for r in recs]
    per = [tickets(kinds[i], int(r["units"])) for i, r in enumerate(recs)]
    owner = np.repeat(np.arange(len(recs)), per)
    assert len(owner) == total
    rec_left = np.array(per)
    done = np.zeros(len(sizes), np.int64)
    rng = np.random.default_rng(workers * 1000 + P)
    head = 0
    held = [None] * workers   # ticket each worker holds
    for w in range(workers):
        if head < total:
            held[w] = head
            head += 1
    finished = 0
    stalls = 0
    while finished < total:
        w = int(rng.integers(workers))
        t = held[w]
        if t is None:
            continue
        r = owner[t]
        b = int(recs[r]["mat"])
        if done[b] < recs[r]["need"]:
            stalls += 1
            # some held ticket must be able to run (no deadlock)
            assert any(h is not None and done[int(recs[owner[h]]["mat"])] >= recs[owner[h]]["need"]
                       for h in held), "every held ticket waits"
            continue
        # every earlier phase of this matrix is complete
        earlier = [i for i in range(r) if int(recs[i]["mat"]) == b]
        assert all(rec_left[i] == 0 for i in earlier)
        rec_left[r] -= 1
        done[b] += 1
        finished += 1
        held[w] = head if head < total else None
        head += 1 if head < total else 0
    assert (rec_left == 0).all()


def test_plan_refuses_mfma_and_bad_sizes(lib):
    with pytest.raises(binding.MpdetError) as e:
        binding.batched_plan([10, 20], 128, "mfma")
    assert e.value.status == binding.MPDET_ENOTSUP
    with pytest.raises(binding.MpdetError) as e:
        binding.batched_plan([10, 0], 8, "valu")
    assert e.value.status == binding.MPDET_EINVAL
