"""Shared templates against per-instance copies (CrowdSplat §2, the paragraph
on reusing every Gaussian parameter but the means; Tab. 1): the unshared
layout draws the same image, and the memory report shows that what an
instance costs does not depend on its template's attribute size unless the
instance holds its own copy."""
import numpy as np
import pytest

from paper_2501_17792_amd import synth

pytestmark = pytest.mark.gpu


def _scene(sh_degree, n_inst=8, n_gauss=20000):
    templates = [synth.make_template(t, n_gauss, sh_degree, synth.C2_LEVELS) for t in range(3)]
    crowd = synth.make_crowd(100, n_inst, 3, 12.0, 0.3)
    cam = synth.look_at((6.0, 1.7, -3.0), (6.0, 1.0, 8.0), 480, 270)
    return synth.Scene("c2slice", templates, crowd, cam, lod_thresholds=(6.0, 11.0))


def _frame(r, sc):
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    img = r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds, stats=True)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def _copy_bytes(t):
    up = lambda b: (b + 255) // 256 * 256  # noqa: E731  (columns start on 256-byte boundaries)
    n = t.n
    n_sh4 = (3 * (t.sh_degree + 1) ** 2 + 3) // 4
    return 3 * up(16 * n) + up(8 * n) + up(4 * n) + up(16 * n * n_sh4)


def test_materialised_instances_draw_the_same_frame():
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _scene(3)
    for fuse in (False, True):
        r = cs.Renderer(0, fuse=fuse)
        r.upload_templates(sc.templates)
        r.set_crowd(sc.crowd)
        ref = _frame(r, sc)
        m0 = r.memory()
        assert m0["instance_copies"] == 0 and m0["n_copies"] == 0
        r.materialise(True)
        m1 = r.memory()
        want = sum(_copy_bytes(sc.templates[int(t)]) for t in sc.crowd.tid)
        # the copies plus the per-instance template table
        assert want <= m1["instance_copies"] <= want + 1024 * sc.crowd.n
        assert m1["n_copies"] == sc.crowd.n
        img = _frame(r, sc)
        assert np.array_equal(img, ref), fuse
        r.materialise(False)
        assert r.memory()["instance_copies"] == 0
        assert np.array_equal(_frame(r, sc), ref)
        # a frame over a different instance count is refused while copies exist
        r.materialise(True)
        sub = synth.Crowd(tid=sc.crowd.tid[:3], yaw=sc.crowd.yaw[:3], pos=sc.crowd.pos[:3], pose=sc.crowd.pose[:3])
        r.set_crowd(sub)
        with pytest.raises(cs.CrowdSplatError) as e:
            r.select_lod(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds)
        assert e.value.code == cs.CS_ERR_STATE
        r.close()


def test_per_instance_bytes_do_not_depend_on_attribute_size():
    """SH degree 0 against 3 (16 against 196 attribute bytes per Gaussian),
    same geometry: the shared layout's per-instance, per-splat and per-pair
    bytes are equal and only the template store grows; with per-instance
    copies the instance cost grows with the attribute size."""
    from paper_2501_17792_amd import crowdsplat as cs

    mem = {}
    for d in (0, 3):
        sc = _scene(d)
        r = cs.Renderer(0)
        r.upload_templates(sc.templates)
        r.set_crowd(sc.crowd)
        _frame(r, sc)
        shared = r.memory()
        r.materialise(True)
        _frame(r, sc)
        mem[d] = (shared, r.memory(), sc)
        r.close()
    s0, c0, sc0 = mem[0]
    s3, c3, sc3 = mem[3]
    for key in ("per_instance", "per_splat", "per_pair", "workspace", "cap_splats", "cap_pairs"):
        assert s0[key] == s3[key], key
    n_gauss = sum(t.n for t in sc0.templates)
    # the shared store grows by the SH planes only: 12 float4 planes at SH3, 1 at SH0
    assert s3["templates"] - s0["templates"] == n_gauss * 16 * (12 - 1)
    per_inst_0 = c0["instance_copies"] / sc0.crowd.n
    per_inst_3 = c3["instance_copies"] / sc3.crowd.n
    assert per_inst_3 > 3 * per_inst_0
    assert c3["total"] - s3["total"] == c3["instance_copies"]
