"""Pushforward training (surrogate_train.train with rollout > 0), checked on
the CPU with a stand-in network: every input tensor encodes its (trajectory,
frame), so the test can read back which frames the loop fed the network."""
import torch

from paper_2405_02914_amd import surrogate_train as T


class Recorder:
    """Stands in for sur.Surrogate: sur_infer adds 1000 to its previous
    displacement, so a fed-back prediction is recognisable."""

    def __init__(self):
        self.infers, self.steps = [], []

    def sur_set_lr(self, lr):
        self.lr = lr

    def sur_infer(self, depth, pose, prev):
        self.infers.append((depth.clone(), prev.clone()))
        return prev + 1000.0

    def sur_train_step(self, depth, pose, prev, tgt, want_loss=False):
        self.steps.append((depth.clone(), prev.clone(), tgt.clone(), len(self.infers)))
        return 1.0


def dataset(n_traj=5, frames=6, res=2):
    code = torch.arange(n_traj)[:, None] * 100.0 + torch.arange(frames + 1)[None, :]     # t * 100 + k
    depth = code[:, :, None, None].expand(n_traj, frames + 1, res, res).clone()
    disp = code[:, :, None, None, None].expand(n_traj, frames + 1, res, res, 3).clone()
    pose6 = code[:, :, None].expand(n_traj, frames + 1, 6).clone()
    return T.Dataset(depth, disp, pose6, 1.0, 1)


def test_plain_training_feeds_the_recorded_previous_frame():
    net = Recorder()
    T.train(net, dataset(), steps=20, batch=4, stream=None, log=lambda *a, **k: None)
    assert not net.infers
    for depth, prev, tgt, _ in net.steps:
        code = depth[:, 0, 0]
        assert torch.equal(tgt[:, 0, 0, 0], code)
        assert torch.equal(prev[:, 0, 0, 0], code - 1)           # frame k - 1 of the same trajectory


def test_pushforward_feeds_the_networks_own_predictions():
    net = Recorder()
    steps, R, frm = 60, 3, 0.5
    data = dataset()
    T.train(net, data, steps=steps, batch=4, stream=None, log=lambda *a, **k: None, rollout=R, rollout_from=frm)
    seen = set()
    done = 0
    for it, (depth, prev, tgt, n_inf) in enumerate(net.steps):
        r = n_inf - done
        assert r == 0 or it >= frm * steps                        # no roll-out before rollout_from
        assert 0 <= r <= min(R, data.F - 1)
        code = depth[:, 0, 0]
        k = code % 100
        assert torch.equal(tgt[:, 0, 0, 0], code)
        assert bool((k >= r + 1).all())
        # r predictions on from the recorded frame k - 1 - r
        assert torch.equal(prev[:, 0, 0, 0], code - 1 - r + 1000.0 * r)
        for j in range(r):                                        # prediction j takes frame k - r + j's inputs
            d_in, p_in = net.infers[done + j]
            assert torch.equal(d_in[:, 0, 0], code - r + j)
            assert torch.equal(p_in[:, 0, 0, 0], code - 1 - r + 1000.0 * j)
        done = n_inf
        seen.add(r)
    assert seen == set(range(R + 1))
