"""Helpers for the GPU parity tests: run the library's pipeline on a batch
and fetch the per-image pieces (no arithmetic of the method here)."""
import numpy as np


def device():
    import torch
    return torch.device("cuda:0")


def pack_images(images, pitch_pad=0):
    """Pack uint8 images into one flat buffer; returns (buffer, descriptors
    with row_pitch / pixel_offset).  pitch_pad adds bytes to each row."""
    descs, chunks, off = [], [], 0
    for im in images:
        h, w = im.shape
        pitch = (w + pitch_pad + 3) // 4 * 4
        buf = np.zeros((h, pitch), dtype=np.uint8)
        buf[:, :w] = im
        chunks.append(buf.reshape(-1))
        descs.append(dict(height=h, width=w, row_pitch=pitch, pixel_offset=off))
        off += buf.size
    return np.concatenate(chunks) if chunks else np.zeros(0, np.uint8), descs


class Run:
    """budget -> sense -> reconstruct through the C ABI for a list of
    (pixel descriptor, block, subrate, method) entries."""

    def __init__(self, px_host, entries):
        import torch
        import paper_2001_09632_amd as g
        dev = device()
        self.plan = g.Plan(entries)
        self.px = torch.from_numpy(px_host).to(dev)
        n = self.plan.blocks
        self.k = torch.full((n,), -7, dtype=torch.int32, device=dev)
        self.off = torch.full((n,), -7, dtype=torch.int64, device=dev)
        self.stat = torch.full((n,), -7, dtype=torch.int32, device=dev)
        self.y = torch.full((max(1, self.plan.meas),), float("nan"), dtype=torch.float32, device=dev)
        self.out = torch.full((max(1, self.plan.pixels),), float("nan"), dtype=torch.float32, device=dev)

    def budget(self):
        import paper_2001_09632_amd as g
        g.budget(self.plan, self.px, self.k, self.off, self.stat)
        return self

    def sense(self):
        import paper_2001_09632_amd as g
        g.sense(self.plan, self.px, self.k, self.off, self.y)
        return self

    def reconstruct(self, y=None):
        import paper_2001_09632_amd as g
        g.reconstruct(self.plan, self.y if y is None else y, self.k, self.off, self.out)
        return self

    def encode(self, out=True, precision="fp32"):
        """The one-call encoder (abcs_encode): budget, sense and, with out,
        the decoder's image."""
        import paper_2001_09632_amd as g
        g.encode(self.plan, self.px, self.k, self.off, self.stat, self.y, self.out if out else None,
                 precision=precision)
        return self

    def fetch(self):
        import torch
        torch.cuda.synchronize()
        self.h_k = self.k.cpu().numpy()
        self.h_off = self.off.cpu().numpy()
        self.h_stat = self.stat.cpu().numpy()
        self.h_y = self.y.cpu().numpy()
        self.h_out = self.out.cpu().numpy()
        return self

    def image(self, i):
        d = self.plan.images[i]
        b0 = d["block_offset"]
        B = d["block"]
        nb = (d["cropped_height"] // B) * (d["cropped_width"] // B)
        m0, nm = d["meas_offset"], d["n_meas"]
        o0 = d["out_offset"]
        hc, wc = d["cropped_height"], d["cropped_width"]
        return dict(k=self.h_k[b0:b0 + nb], off=self.h_off[b0:b0 + nb] - m0, stat=self.h_stat[b0:b0 + nb],
                    y=self.h_y[m0:m0 + nm], out=self.h_out[o0:o0 + hc * wc].reshape(hc, wc), desc=d)
