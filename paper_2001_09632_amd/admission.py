"""Admission of encode requests into batches under a device-memory budget.

A serving loop holds a fixed amount of device memory for the outputs of one
batch: y (4 bytes per coefficient), optionally the decoded images (4 bytes
per pixel) and the per-block arrays k, offsets and stat (4 + 8 + 4 bytes per
block).  Requests are admitted in arrival order; a batch closes when the next
request would not fit, so no request waits behind a later one.  A request's
sizes come from the library's own geometry and budget rules
(abcs_image_totals: cropping, M = floor(C_R N), the BBV samples), exactly as
a plan would count them, before any plan is made.
"""
from .api import image_totals

BLOCK_BYTES = 4 + 8 + 4   # k, offsets, stat


class Admission:
    """budget_bytes: device bytes one batch may use for its outputs;
    decode: whether the batch also writes the decoded images."""

    def __init__(self, budget_bytes, decode=True):
        if budget_bytes <= 0:
            raise ValueError("budget_bytes must be positive")
        self.budget = int(budget_bytes)
        self.decode = bool(decode)

    def cost(self, desc):
        """Device bytes of one request's outputs (raises AbcsError for a
        descriptor a plan would reject)."""
        blocks, meas, pixels = image_totals(desc)
        return 4 * meas + (4 * pixels if self.decode else 0) + BLOCK_BYTES * blocks

    def batches(self, descs):
        """Indices of descs grouped into batches in arrival order.  A request
        larger than the whole budget cannot be served: ValueError."""
        out, cur, used = [], [], 0
        for i, d in enumerate(descs):
            c = self.cost(d)
            if c > self.budget:
                raise ValueError(f"request {i} needs {c} bytes, more than the batch budget {self.budget}")
            if cur and used + c > self.budget:
                out.append(cur)
                cur, used = [], 0
            cur.append(i)
            used += c
        if cur:
            out.append(cur)
        return out

    def first_batch(self, descs):
        """The batch that the first of descs opens (what a loop serves now)."""
        out, used = [], 0
        for i, d in enumerate(descs):
            c = self.cost(d)
            if out and used + c > self.budget:
                break
            if c > self.budget:
                raise ValueError(f"request {i} needs {c} bytes, more than the batch budget {self.budget}")
            out.append(i)
            used += c
        return out
