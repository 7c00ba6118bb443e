"""Host-side logic of bench.py (CPU): the one-GPU guard and the lookup of the
committed HBM-traffic record, which is valid only for the kernel sources it
was measured on."""

import json
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""   # no JSON line


def _record():
    text = open(bench.TRAFFIC_FILE).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    assert m, "the traffic summary carries a JSON record"
    return json.loads(m.group(1))


def test_traffic_record_is_used_only_for_its_sources(monkeypatch):
    rec = _record()
    key = "bp_brick_kernel/f32"
    assert key in rec
    r = rec[key]
    assert r["hbm_bytes_per_launch"] == r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"]
    # sources as measured: the record's bytes
    monkeypatch.setattr(bench, "source_hash", lambda kernel: r["source_hash"])
    assert bench.measured_traffic("bp_brick_kernel", "f32") == r["hbm_bytes_per_launch"]
    # any other sources: no traffic figure
    monkeypatch.setattr(bench, "source_hash", lambda kernel: "0" * 16)
    assert bench.measured_traffic("bp_brick_kernel", "f32") is None
    # a kernel or precision without a record
    assert bench.measured_traffic("bp_brick_kernel", "bf16") is None


def test_source_hash_covers_every_listed_file(monkeypatch):
    # changing any byte of any listed source changes the hash
    h0 = bench.source_hash("bp_brick_kernel")
    src = os.path.join(ROOT, "paper_2609_30166_amd", "csrc")
    for f in bench.KERNEL_SOURCES["bp_brick_kernel"]:
        assert os.path.exists(os.path.join(src, f))
    real_open = open

    def fake_open(path, mode="r", *a, **k):
        fh = real_open(path, mode, *a, **k)
        if path.endswith("ray_common.h") and "b" in mode:
            data = fh.read() + b" "
            fh.close()
            import io
            return io.BytesIO(data)
        return fh

    monkeypatch.setattr("builtins.open", fake_open)
    assert bench.source_hash("bp_brick_kernel") != h0


def test_unet_flop_count_matches_torch_flop_counter():
    """The FLOPs behind the reported U-Net rate, counted independently: torch's
    flop counter over the same network written with plain torch operators
    (3x3x3 same-padded convolutions, 2x2x2 stride-2 transposed convolutions,
    a 1x1x1 head; pooling and concatenation cost no FLOPs)."""
    import torch
    import torch.nn.functional as F
    from torch.utils.flop_counter import FlopCounterMode

    from paper_2609_30166_amd.unet import LAYERS

    n = 8
    w = {name: torch.rand(cout, cin, 3, 3, 3) if kind == "conv" else torch.rand(cin, cout, 2, 2, 2)
         for name, kind, cin, cout in LAYERS}

    def conv(name, t):
        return F.relu(F.conv3d(t, w[name], padding=1))

    def up(name, t):
        return F.conv_transpose3d(t, w[name], stride=2)

    x = torch.rand(1, 1, n, n, n)
    with FlopCounterMode(display=False) as fc:
        e1 = conv("e1b", conv("e1a", x))
        e2 = conv("e2b", conv("e2a", F.max_pool3d(e1, 2)))
        b = conv("bnb", conv("bna", F.max_pool3d(e2, 2)))
        d2 = conv("d2b", conv("d2a", torch.cat([up("up2", b), e2], 1)))
        d1 = conv("d1b", conv("d1a", torch.cat([up("up1", d2), e1], 1)))
        F.conv3d(d1, torch.rand(1, 16, 1, 1, 1))
    assert fc.get_total_flops() == bench.unet_flops(n)
