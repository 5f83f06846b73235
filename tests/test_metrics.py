"""The JSON-lines metrics writer: per-ligand acceptances as ratios (None
where nothing was tried), round trips and non-finite moves from the
counters, the caller's figures on every line."""
import json

import numpy as np

from paper_1507_03703_amd import metrics as M


class FakeContext:
    def get_stats(self, ligand_id):
        return dict(hmc_acc=np.array([3, 0]), hmc_try=np.array([4, 0]),
                    ex_acc=np.array([1]), ex_try=np.array([2]),
                    nonfinite=5 + ligand_id)

    def get_round_trips(self, ligand_id):
        return 7 * ligand_id


def test_lines_carry_counters_and_figures(tmp_path):
    path = tmp_path / "m.jsonl"
    log = M.MetricsLog(str(path))
    log.record(FakeContext(), [0, 2], workload="toy", atom_evals_per_s=1.5e9)
    log.record(FakeContext(), [1], ess_per_s=12.0)
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    assert [l["ligand"] for l in lines] == [0, 2, 1]
    first = lines[0]
    assert first["hmc_acceptance"] == [0.75, None]
    assert first["exchange_acceptance"] == [0.5]
    assert first["hmc_tries"] == 4 and first["exchange_tries"] == 2
    assert first["round_trips"] == 0 and lines[1]["round_trips"] == 14
    assert first["nonfinite"] == 5 and lines[2]["nonfinite"] == 6
    assert first["workload"] == "toy" and first["atom_evals_per_s"] == 1.5e9
    assert "workload" not in lines[2] and lines[2]["ess_per_s"] == 12.0
    assert all(isinstance(l["time"], float) for l in lines)
