"""QAOA angle optimisation on the adjoint gradient.

The paper tunes the QAOA angles with an external derivative-free optimiser
(Sec. QAOA / Max-Cut). Here the optimiser is a host-side Adam ascent that
consumes the batched forward+adjoint pass: every iteration is one
`tn_batch_grad` over all starting points at once, and the Adam update runs as
a few elementwise tensor operations on the same device.
"""


def adam_maximize(value_and_grad, x0, steps=200, lr=0.05, betas=(0.9, 0.999), eps=1e-8):
    """Maximise f independently for every row of x0 (S x P) by Adam ascent.

    value_and_grad(x) -> (f of shape (S,), g of shape (S, P)), tensors on x's
    device and dtype. Returns (x_best, f_best, trace): per row the best point
    seen and its value, and the per-iteration maximum over rows (a tensor of
    steps + 1 entries, left on the device)."""
    import torch
    x = x0.detach().clone()
    m = torch.zeros_like(x)
    v = torch.zeros_like(x)
    f, g = value_and_grad(x)
    best_f, best_x = f.clone(), x.clone()
    trace = [f.max()]
    b1, b2 = betas
    for t in range(1, steps + 1):
        m.mul_(b1).add_(g, alpha=1 - b1)
        v.mul_(b2).addcmul_(g, g, value=1 - b2)
        x = x + lr * (m / (1 - b1 ** t)) / ((v / (1 - b2 ** t)).sqrt() + eps)
        f, g = value_and_grad(x)
        better = f > best_f
        best_f = torch.where(better, f, best_f)
        best_x = torch.where(better[:, None], x, best_x)
        trace.append(f.max())
    return best_x, best_f, torch.stack(trace)


def maxcut_optimize(model, x0, steps=200, lr=0.05):
    """Adam ascent of <C>(gamma, beta) for a `qaoa.MaxCut` model from the
    starting angle sets x0 (S x 2p, at most the model's max_sets rows)."""
    import torch
    x0 = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
    return adam_maximize(model.value_and_grad, x0, steps=steps, lr=lr)
