"""The README's Python quick start runs as written (GPU)."""
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.gpu
def test_readme_quick_start_runs():
    text = (ROOT / "README.md").read_text()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert len(blocks) == 1
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    borth, info, inf, infos = env["borth"], env["info"], env["inf"], env["infos"]
    assert info.status == 0 and inf.status == 0 and all(i.status == 0 for i in infos)
    Q, Qh = env["Q"], env["Qh"]
    assert Q.shape[1] == 4 and Qh.shape == (4_000_000, 4)
    assert isinstance(borth.ArgumentError("x"), ValueError)
