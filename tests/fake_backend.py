"""A serving backend that decodes with the CPU oracle (test infrastructure): it lets the
scheduler's admission, budget and batching logic run without a GPU."""
import numpy as np

import oracle


class OracleBackend:
    def __init__(self, infos, crc_bits, n_slots=2, delay_polls=2):
        self.infos = infos
        self.crc = crc_bits
        self.slots = [{"busy": False, "batch": None, "polls": 0} for _ in range(n_slots)]
        self.delay = delay_polls
        self.max_concurrent = 0

    def free_slots(self):
        return [i for i, s in enumerate(self.slots) if not s["busy"]]

    def submit(self, slot, reqs):
        s = self.slots[slot]
        assert not s["busy"]
        for r in reqs:
            pay, st, _ = oracle.scs_decode_batch(oracle.F32, self.infos[r.code], self.crc, r.D, r.L, r.llr)
            r.payload, r.status = pay, st
        s.update(busy=True, batch=reqs, polls=0)
        self.max_concurrent = max(self.max_concurrent, sum(x["busy"] for x in self.slots))

    def done(self, slot):
        s = self.slots[slot]
        if not s["busy"]:
            return False
        s["polls"] += 1
        return s["polls"] > self.delay

    def collect(self, slot):
        s = self.slots[slot]
        reqs = s["batch"]
        s.update(busy=False, batch=None)
        return reqs
