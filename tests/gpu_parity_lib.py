"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on the same seeded inputs and compare."""
import math
import sys

import numpy as np

from paper_2110_06635_amd import synth

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_device_scene(A, ctx, s, dtype="f32", prepare=True, block=0, seed=7):
    import torch
    raw, widened = synth.storage(s.feat, dtype)
    pos = torch.from_numpy(np.ascontiguousarray(s.pos)).cuda()
    if dtype == "f32":
        feat = torch.from_numpy(raw).cuda()
    else:
        feat = torch.from_numpy(raw.view(np.int16)).cuda().view(A.TORCH_STORAGE[A.DTYPES[dtype]])
    code = A.DTYPES[dtype]
    if prepare:
        scene = A.Scene.prepare(ctx, pos, feat, code, block=block, seed=seed)
    else:
        scene = A.Scene.identity(pos, feat, code)
    return scene, widened


def gpu_forward(A, ctx, scene, s, alpha=None, flags=0):
    import torch
    alpha = s.alpha if alpha is None else alpha
    fr = A.render_forward(ctx, scene, s.cams, s.layers, alpha=alpha, flags=flags, background=s.bg())
    torch.cuda.synchronize()
    return fr


def frame_numpy(fr):
    return (fr.keys.cpu().numpy().view(np.uint64), fr.counts.cpu().numpy(), fr.images.cpu().numpy())


def compare_forward(fr, ref, rtol=1e-5, scale=1.0):
    keys, counts, images = frame_numpy(fr)
    nk = int(np.sum(keys != ref["keys"]))
    assert nk == 0, f"{nk} keys differ"
    nc = int(np.sum(counts != ref["counts"]))
    assert nc == 0, f"{nc} counts differ"
    err = np.abs(images.astype(np.float64) - ref["images64"])
    bound = rtol * np.abs(ref["images64"]) + 1e-7 * scale
    bad = err > bound
    assert not bad.any(), f"{int(bad.sum())} image values off, worst rel {float(np.max(err / (np.abs(ref['images64']) + 1e-30))):.3g}"
    return float(np.max(err / (np.abs(ref["images64"]) + 1e-12 * scale)))


def to_user_order(orig, arr, axis=0):
    out = np.empty_like(arr)
    if axis == 0:
        out[orig] = arr
    else:
        out[:, orig] = arr
    return out


def compare_backward(scene, got, ref, tol_feat=1e-5, tol_pos=1e-4, tol_cam=1e-5):
    dfeat, dpos, dpose, dintr = [t.cpu().numpy() for t in got]
    orig = scene.orig.cpu().numpy()
    dfeat = to_user_order(orig, dfeat, 0)
    dpos = to_user_order(orig, dpos, 1)
    report = {}

    def chk(name, g, r, s, tol):
        err = np.abs(g.astype(np.float64) - r)
        lim = tol * s + 1e-12
        bad = err > lim
        assert not bad.any(), (f"{name}: {int(bad.sum())} of {bad.size} beyond {tol}*S; "
                               f"worst err/S {float(np.max(err / (s + 1e-30))):.3g}")
        report[name] = float(np.max(err / (s + 1e-30))) if err.size else 0.0

    chk("dfeat", dfeat, ref["dfeat"], ref["dfeat_abs"], tol_feat)
    chk("dpos", dpos, ref["dpos"], ref["dpos_abs"], tol_pos)
    chk("dpose", dpose, ref["dpose"], ref["dpose_abs"], tol_cam)
    chk("dintr", dintr, ref["dintr"], ref["dintr_abs"], tol_cam)
    return report


def check_visibility(fr, s):
    """The forward's blend-set bits against the bit-exact counts: for every
    view and layer, the number of points with bit l set equals the sum of
    the layer's counts, and no bit at or above L is set."""
    vis = fr.visible.cpu().numpy()
    counts = fr.counts.cpu().numpy()
    for v, cam in enumerate(s.cams):
        assert not np.any(vis[v] >> s.layers), "bits above the layer count"
        for l in range(s.layers):
            o = int(fr.offsets[v, l])
            npx = (cam.width >> l) * (cam.height >> l)
            got = int(np.count_nonzero((vis[v] >> l) & 1))
            want = int(counts[o:o + npx].sum(dtype=np.int64))
            assert got == want, f"view {v} layer {l}: {got} points flagged, counts sum to {want}"
    return True


def run_case(A, ctx, O, s, dtype="f32", prepare=True, flags=0, grad_seed=99, backward=True, alpha=None,
             normals=None, radius=None, beta=None, gamma=1.5, visibility=True):
    """Forward (+ backward) on GPU and oracle; returns reports.  normals
    [n,3], radius [n] and beta [n] (caller's order) go with the culling and
    discarding flags.  visibility: the forward records the blend-set bits
    and the backward reads them (False: the backward re-tests every point)."""
    import torch
    alpha = s.alpha if alpha is None else alpha
    scene, widened = to_device_scene(A, ctx, s, dtype, prepare)
    if normals is not None:
        scene.set_normals(ctx, torch.from_numpy(np.ascontiguousarray(normals, np.float32)).cuda())
    if beta is not None:
        scene.set_discard(ctx, torch.from_numpy(np.ascontiguousarray(beta, np.float32)).cuda(),
                          torch.from_numpy(np.ascontiguousarray(radius, np.float32)).cuda())
    opt = dict(flags=flags, normals=normals, radius=radius, beta=beta, gamma=gamma)
    fr = A.render_forward(ctx, scene, s.cams, s.layers, alpha=alpha, flags=flags, background=s.bg(), gamma=gamma,
                          record_visibility=visibility)
    torch.cuda.synchronize()
    ref = O.forward(s.pos, widened, s.cams, s.layers, alpha=alpha, background=s.bg(), want64=True, **opt)
    scale = max(1.0, float(np.max(np.abs(widened))) if widened.size else 1.0)
    rep = {"image_rel": compare_forward(fr, ref, scale=scale)}
    if visibility and s.n > 0:
        rep["visible_bits"] = check_visibility(fr, s)
    if backward:
        total = fr.pixels
        G = synth.upstream_grad(total * s.c, grad_seed)
        g = torch.from_numpy(G).cuda()
        got = A.render_backward(ctx, scene, fr, g, alpha=alpha, flags=flags, background=s.bg(), gamma=gamma)
        torch.cuda.synchronize()
        rb = O.backward(s.pos, widened, s.cams, s.layers, G, alpha=alpha, background=s.bg(), **opt)
        rep.update(compare_backward(scene, got, rb))
    return rep
