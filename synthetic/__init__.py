"""Seeded synthetic inputs shared by the oracle-side tests and the product's
tests and benchmark.  Holds no arithmetic of the method: it only draws random
numbers with the shapes and distributions of the workloads.

Recipes (all on the CPU, ``torch.Generator().manual_seed(seed)``):

* single-channel cross-correlation: image (oh+fh-1) x (ow+fw-1) then filter
  fh x fw, both FP32 uniform[0, 1), drawn in that order;
* multi-channel convolution: activations [n][h][w][c_in] then weights
  [c_out][fh][fw][c_in], FP32 N(0, 1) rounded to nearest-even BF16;
* serving mix: Poisson arrivals (exponential gaps) at a fixed rate; square
  output side round(exp(U[ln 128, ln 4096])); filter side uniform from
  {3, 5, 9, 17}; 30 % of requests BF16 multi-channel (N=1, C_in=C_out=32,
  same padding), the rest FP32 single-channel valid.
"""
import math

import torch


def xcorr_inputs(out_h, out_w, fh, fw, seed=0):
    g = torch.Generator().manual_seed(seed)
    image = torch.rand(out_h + fh - 1, out_w + fw - 1, generator=g, dtype=torch.float32)
    filt = torch.rand(fh, fw, generator=g, dtype=torch.float32)
    return image, filt


def conv_inputs(n, h, w, c_in, c_out, fh, fw, seed=0):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(n, h, w, c_in, generator=g, dtype=torch.float32).to(torch.bfloat16)
    wt = torch.randn(c_out, fh, fw, c_in, generator=g, dtype=torch.float32).to(torch.bfloat16)
    return x, wt


def integer_inputs(out_h, out_w, fh, fw, lo=-4, hi=5, seed=0):
    """Small integer-valued FP32 data: every product and sum is exact in FP32
    and FP64 for the sizes used in tests."""
    g = torch.Generator().manual_seed(seed)
    image = torch.randint(lo, hi, (out_h + fh - 1, out_w + fw - 1), generator=g).to(torch.float32)
    filt = torch.randint(lo, hi, (fh, fw), generator=g).to(torch.float32)
    return image, filt


def serving_requests(n_req, rate_hz, seed=0, frac_multi=0.3, c_multi=32,
                     side_lo=128, side_hi=4096, filters=(3, 5, 9, 17)):
    """List of dicts {t_arrive, kind ('xcorr_f32' | 'conv_bf16'), side, f, c}."""
    g = torch.Generator().manual_seed(seed)
    u = torch.rand(n_req, 4, generator=g, dtype=torch.float64)
    t = 0.0
    out = []
    for k in range(n_req):
        t += -math.log(max(1.0 - float(u[k, 0]), 1e-300)) / rate_hz
        side = int(round(math.exp(math.log(side_lo) + float(u[k, 1]) * (math.log(side_hi) - math.log(side_lo)))))
        f = filters[min(int(float(u[k, 2]) * len(filters)), len(filters) - 1)]
        multi = float(u[k, 3]) < frac_multi
        out.append(dict(t_arrive=t, kind="conv_bf16" if multi else "xcorr_f32", side=side, f=f,
                        c=c_multi if multi else 1))
    return out
